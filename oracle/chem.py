"""Oracle, chemical-reaction workload: the slow-fast SDE of Sec. 2.1.2 with
multiplicative noise, its macroscopic model (Sec. 2.2.1, the chemical
reactions example) and the finite-volume coarse propagator of Sec. 2.2.2 with
a state-dependent effective diffusion.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Readings where the paper is silent or at odds with itself (each listed in the
design notes):
  R1 drifts: the chemical-Langevin drifts of the reactions whose summed
     propensities are 2D and 2E (see oracle.c): -dF/dx = k4 y - k5 x and
     -dG/dy = k0 - k1 y + k2 y(y-1) - k3 y(y-1)(y-2).  The printed signs of
     the k1, k2, k3, k5 terms give drifts with no stable state.
  R2 k3: the default table value is read as 0.666e-5.  With 0.666e-6 the fast
     drift has a single root near y = 7000: no bistability, and a fast mean
     (hence a slow equilibrium k4 ybar/k5) far outside the grid [0, 600]; with
     0.666e-5 its roots are near 105, 211 and 408 (two stable states around an
     unstable one), the bistable fast variable that the experiments describe.
     The rates are parameters; only the default takes this reading.
  R3 D and E enter the square roots as max(., 0).
  R4 initial law: lognormal with the stated mean and standard deviation
     (log X0 ~ N(log m - s^2/2, s^2), s^2 = log(1 + sd^2/m^2)).
  R5 ybar: the trapezoidal rule on the uniform grid of [0, 1000] with spacing
     1e-2, both for the inner integral (running sum from 0) and for the
     normalised mean of phi(y) = exp(int_0^y b/E ds)/E(y).
  R6 coarse model: by eq. (Fbar)/(Dbar) with phi independent of x,
     Fbar'(x) = -(k4 ybar - k5 x) and Dbar(x) = (k4 ybar + k5 x)/2;
     rho_inf(x) = exp(-int_0^x Fbar'/Dbar ds)/Dbar(x) as in Sec. 2.2.2; the
     edge coefficients a_i = Dbar(x_i) rho_inf(x_i)/(tau_x h) (zero at the
     two grid ends) and g_i = h rho_inf(m_i) of the uniform-grid scheme.
"""
import ctypes

import numpy as np
import scipy.integrate as _si
import scipy.linalg as _sla

from . import particles as _particles

K_DEFAULT = (60.0, 1.0, 4.8e-3, 0.666e-5, 0.833, 1.0)


class _Chem(ctypes.Structure):
    _fields_ = [("tau_x", ctypes.c_double), ("eps", ctypes.c_double), ("k", ctypes.c_double * 6),
                ("x0_mean", ctypes.c_double), ("x0_sd", ctypes.c_double),
                ("y0_mean", ctypes.c_double), ("y0_sd", ctypes.c_double)]


class Chem:
    """Parameters of the chemical-reaction system (Table 1 defaults, with the
    reading R2 of k3)."""

    def __init__(self, tau_x=25.0, eps=2.5e-2, k=K_DEFAULT, x0=(100.0, 20.0), y0=(100.0, 20.0)):
        self.tau_x, self.eps = float(tau_x), float(eps)
        self.k = tuple(float(v) for v in k)
        self.x0, self.y0 = tuple(x0), tuple(y0)
        self.d = 1

    def c(self):
        s = _Chem()
        s.tau_x, s.eps = self.tau_x, self.eps
        for i in range(6):
            s.k[i] = self.k[i]
        s.x0_mean, s.x0_sd = self.x0
        s.y0_mean, s.y0_sd = self.y0
        return s


def _lib():
    L = _particles.lib()
    if not getattr(L, "_chem_ready", False):
        P = ctypes.POINTER
        u32, u64, i64, dbl, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.or_chem_init.argtypes = [P(_Chem), u64, u32, i64, vp, vp]
        L.or_chem_em.argtypes = [P(_Chem), u64, u32, i64, i64, i64, i64, dbl, vp, vp]
        L.or_chem_init.restype = None
        L.or_chem_em.restype = None
        L._chem_ready = True
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def init_ensemble(c, seed, inst, n):
    """Initial ensemble (R4): x[n], y[1][n]."""
    x = np.zeros(n)
    y = np.zeros((1, n))
    _lib().or_chem_init(ctypes.byref(c.c()), seed, inst, n, _ptr(x), _ptr(y))
    return x, y


def em_propagate(c, seed, inst, x, y, m_begin, m_end, dt, p0=0):
    """Euler-Maruyama over global steps [m_begin, m_end); returns new (x, y)."""
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    y = np.array(y, dtype=np.float64, copy=True, order="C").reshape(1, -1)
    _lib().or_chem_em(ctypes.byref(c.c()), seed, inst, p0, x.shape[0], m_begin, m_end, dt, _ptr(x), _ptr(y))
    return x, y


# --------------------------------------------------------------------------
# Macroscopic model.
# --------------------------------------------------------------------------
def fast_drift(c, y):
    """b(y) = -dG/dy (R1)."""
    k0, k1, k2, k3 = c.k[:4]
    y = np.asarray(y, dtype=np.float64)
    return k0 - k1 * y + k2 * y * (y - 1.0) - k3 * y * (y - 1.0) * (y - 2.0)


def fast_diffusion(c, y):
    """E(y), eq. (E_Bruna)."""
    k0, k1, k2, k3 = c.k[:4]
    y = np.asarray(y, dtype=np.float64)
    return 0.5 * (k0 + k1 * y + k2 * y * (y - 1.0) + k3 * y * (y - 1.0) * (y - 2.0))


def fast_density(c, y_max=1000.0, dy=1e-2):
    """Nodes y_j = j dy and phi(y_j) / max phi, the equilibrium density
    phi(y) ~ exp(-int_0^y G'(s)/E(s) ds)/E(y) of the fast variable, the inner
    integral by the trapezoidal rule (R5)."""
    n = int(round(y_max / dy))
    y = dy * np.arange(n + 1)
    r = fast_drift(c, y) / fast_diffusion(c, y)
    inner = np.concatenate([[0.0], np.cumsum(0.5 * (r[1:] + r[:-1]) * dy)])
    logphi = inner - np.log(fast_diffusion(c, y))
    return y, np.exp(logphi - logphi.max())


def mean_fast(c, y_max=1000.0, dy=1e-2):
    """ybar = int y phi dy / int phi dy by the trapezoidal rule (R5)."""
    y, phi = fast_density(c, y_max, dy)
    w = np.full(len(y), dy)
    w[0] = w[-1] = 0.5 * dy
    return float(np.sum(w * phi * y) / np.sum(w * phi))


def effective(c, ybar):
    """Fbar'(x) and Dbar(x) of eq. (Fbar)/(Dbar) (R6)."""
    k4, k5 = c.k[4], c.k[5]
    return (lambda x: -(k4 * ybar - k5 * x)), (lambda x: 0.5 * (k4 * ybar + k5 * x))


def log_rho_inf_ratio(c, ybar, xa, xb):
    """log(rho_inf(xa)/rho_inf(xb)) from the definition of rho_inf (Sec. 2.2.2):
    log(Dbar(xb)/Dbar(xa)) - int_xb^xa Fbar'(s)/Dbar(s) ds."""
    dF, Db = effective(c, ybar)
    val, _ = _si.quad(lambda s: dF(s) / Db(s), xb, xa, epsabs=1e-14, epsrel=1e-13, limit=200)
    return float(np.log(Db(xb) / Db(xa)) - val)


def fv_generator(grid, c, ybar):
    """Generator A of d rho/dt = A rho (Sec. 2.2.2 on the uniform grid) and
    the discrete equilibrium g (A g = 0), for the coarse model R6:
      d rho_i/dt = a_{i+1} (rho_{i+1}/g_{i+1} - rho_i/g_i)
                 - a_i (rho_i/g_i - rho_{i-1}/g_{i-1}),
    a_i = Dbar(x_i) rho_inf(x_i)/(tau_x h) at interior edges, 0 at the ends,
    g_i = h rho_inf(m_i).  Every coefficient a_i/g_j is formed from the ratio
    rho_inf(x_i)/rho_inf(m_j) of two neighbouring points."""
    _, Db = effective(c, ybar)
    I, h = grid.n, grid.h
    e, m = grid.edges, grid.mids
    A = np.zeros((I, I))
    for i in range(1, I):  # edge i between cells i-1 and i
        base = Db(e[i]) / (c.tau_x * h * h)
        to_left = base * np.exp(log_rho_inf_ratio(c, ybar, e[i], m[i - 1]))   # a_i / g_{i-1}
        to_right = base * np.exp(log_rho_inf_ratio(c, ybar, e[i], m[i]))      # a_i / g_i
        A[i - 1, i - 1] -= to_left
        A[i, i - 1] += to_left
        A[i, i] -= to_right
        A[i - 1, i] += to_right
    logg = np.zeros(I)
    for i in range(1, I):
        logg[i] = logg[i - 1] + log_rho_inf_ratio(c, ybar, m[i], m[i - 1])
    return A, np.exp(logg - logg.max())


class Propagator:
    """E(tau) = exp(A tau) of the chemical coarse model, by the library matrix
    exponential (Pade scaling-and-squaring)."""

    def __init__(self, grid, c, ybar=None):
        self.ybar = mean_fast(c) if ybar is None else ybar
        self.A, self.g = fv_generator(grid, c, self.ybar)

    def expm(self, tau):
        return _sla.expm(self.A * tau)
