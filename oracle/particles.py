"""Oracle, particle level: noise, initial ensemble, Euler-Maruyama, tangents.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Thin ctypes wrappers around the plain C loops of ``oracle.c`` (built by
``oracle/build.py``).  See that file for the passages of the paper each loop
follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class _Sde(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("lambda_", ctypes.c_double), ("eps", ctypes.c_double),
                ("beta", ctypes.c_double), ("c3", ctypes.c_double), ("c1", ctypes.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        u32, u64, i64, i32, dbl = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64,
                                   ctypes.c_int, ctypes.c_double)
        vp = ctypes.c_void_p
        L.or_philox.argtypes = [vp, vp, vp]
        L.or_blocks.argtypes = [u64, u32, u32, u32, i64, i64, u32, vp]
        L.or_normals.argtypes = [u64, u32, u32, u32, i64, i64, i32, vp]
        L.or_box_muller.argtypes = [vp, vp, vp]
        L.or_coupling.argtypes = [u64, u32, i32, vp]
        L.or_instance_params.argtypes = [u64, u32, P(dbl), P(dbl), P(i64), P(i32)]
        L.or_init_ensemble.argtypes = [P(_Sde), vp, u64, u32, i64, vp, vp]
        L.or_em_propagate.argtypes = [P(_Sde), vp, u64, u32, i64, i64, i64, i64, dbl, vp, vp]
        L.or_em_propagate_f32noise.argtypes = L.or_em_propagate.argtypes
        L.or_box_muller_f32.argtypes = [vp, vp, vp]
        L.or_em_tangent.argtypes = [P(_Sde), u64, u32, i64, i64, dbl, vp, vp, vp, vp]
        for f in ("or_philox", "or_blocks", "or_normals", "or_box_muller", "or_box_muller_f32", "or_coupling",
                  "or_instance_params", "or_init_ensemble", "or_em_propagate", "or_em_propagate_f32noise",
                  "or_em_tangent"):
            getattr(L, f).restype = None
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Sde:
    """Parameters of the slow-fast SDE (Sec. 2.1.1 with tau_x = 1, D = E = 1/beta)."""

    def __init__(self, lam=1.0, eps=0.1, beta=2.0, c3=1.0, c1=-1.0, d=1, a=None):
        self.lam, self.eps, self.beta, self.c3, self.c1, self.d = lam, eps, beta, c3, c1, d
        self.a = None if a is None else np.ascontiguousarray(a, dtype=np.float64)

    def c(self):
        return _Sde(self.d, self.lam, self.eps, self.beta, self.c3, self.c1)

    def abar(self):
        return 1.0 if self.a is None else float(np.mean(self.a))


def philox(ctr, key):
    """One Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def blocks(seed, inst, tag, m, p0, n, j=0):
    out = np.zeros((n, 4), dtype=np.uint32)
    lib().or_blocks(seed, inst, tag, m, p0, n, j, _ptr(out))
    return out


def normals(seed, inst, tag, m, p0, n, n_norm):
    """Standard normals out[p][k] of stream (tag, step m) for particles p0..p0+n-1."""
    out = np.zeros((n, n_norm), dtype=np.float64)
    lib().or_normals(seed, inst, tag, m, p0, n, n_norm, _ptr(out))
    return out


def _pairs(fn, words):
    w = np.ascontiguousarray(np.atleast_2d(words), dtype=np.uint32)
    z = np.zeros((len(w), 2), dtype=np.float64)
    for k in range(len(w)):
        fn(w[k].ctypes.data_as(ctypes.c_void_p), z[k].ctypes.data_as(ctypes.c_void_p),
           ctypes.c_void_p(z[k].ctypes.data + 8))
    return z[:, 0], z[:, 1]


def box_muller(words):
    """Normal pair of each block of words (rows of 4 x u32) -> (z0, z1)."""
    return _pairs(lib().or_box_muller, words)


def box_muller_f32(words):
    """The single-precision propagator's normal pair of each block (its
    24- and 28-bit uniforms, transformed in double precision)."""
    return _pairs(lib().or_box_muller_f32, words)


def coupling(seed, inst, d):
    a = np.zeros(d, dtype=np.float64)
    lib().or_coupling(seed, inst, d, _ptr(a))
    return a


def instance_params(seed, inst):
    eps, lam = ctypes.c_double(), ctypes.c_double()
    n, k = ctypes.c_int64(), ctypes.c_int()
    lib().or_instance_params(seed, inst, ctypes.byref(eps), ctypes.byref(lam),
                             ctypes.byref(n), ctypes.byref(k))
    return eps.value, lam.value, n.value, k.value


def init_ensemble(sde, seed, inst, n):
    """Initial ensemble: x[n], y[d][n]."""
    x = np.zeros(n, dtype=np.float64)
    y = np.zeros((sde.d, n), dtype=np.float64)
    a = sde.a
    lib().or_init_ensemble(ctypes.byref(sde.c()), None if a is None else _ptr(a), seed, inst, n,
                           _ptr(x), _ptr(y))
    return x, y


def em_propagate(sde, seed, inst, x, y, m_begin, m_end, dt, p0=0, f32_noise=False):
    """Euler-Maruyama over global steps [m_begin, m_end); returns new (x, y).
    f32_noise: the normals of the single-precision propagator, the scheme
    still in double precision."""
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    y = np.array(y, dtype=np.float64, copy=True, order="C").reshape(sde.d, -1)
    n = x.shape[0]
    a = sde.a
    fn = lib().or_em_propagate_f32noise if f32_noise else lib().or_em_propagate
    fn(ctypes.byref(sde.c()), None if a is None else _ptr(a), seed, inst, p0, n, m_begin, m_end, dt, _ptr(x),
       _ptr(y))
    return x, y


def em_tangent(sde, seed, inst, n, m_end, dt):
    """Forward-mode pathwise tangents of (X, Y) at step m_end w.r.t.
    theta = (lambda, eps, beta, c3), from the initial ensemble, d = 1, a = 1."""
    assert sde.d == 1 and sde.a is None
    x = np.zeros(n)
    y = np.zeros(n)
    dx = np.zeros((4, n))
    dy = np.zeros((4, n))
    lib().or_em_tangent(ctypes.byref(sde.c()), seed, inst, n, m_end, dt,
                        _ptr(x), _ptr(y), _ptr(dx), _ptr(dy))
    return x, y, dx, dy
