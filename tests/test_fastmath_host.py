"""The FP64 helpers of the Box-Muller transform (table-based -2 ln u, sqrt,
and sin/cos of pi t from the bit fields of a block) against long-double C
library values and against the oracle's transform, on the host build of the
same source (the device build swaps only the reciprocal-sqrt seed and
frexp for their hardware instructions)."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import particles as OP

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1912_09240_amd", "csrc")
LD = np.longdouble
PI_LD = LD("3.14159265358979323846264338327950288")


@pytest.fixture(scope="module")
def fm():
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    so = os.path.join(d, "fm.so")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                           "-I", CSRC, "-I", os.path.join(os.path.dirname(HERE), "include"),
                           os.path.join(HERE, "fastmath_host.hip"), "-o", so],
                          stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(so)
    for f in (L.fm_neg2_ln, L.fm_sqrt_pos, L.fm_sqrt_positive):
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
    L.fm_sincos_cell.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_long]
    L.fm_normal_pair.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_long]
    return L


def _ulps(a, ref):
    return np.abs(a - ref) / np.spacing(np.abs(ref).astype(np.float64))


def _grid_u(k):
    """u = (k + 1/2) 2^-52, the values the transform sees."""
    return (k.astype(np.float64) + 0.5) * 2.0 ** -52


def test_neg2_ln(fm):
    rng = np.random.default_rng(0)
    k = np.concatenate([
        rng.integers(0, 2 ** 52, 400_000, dtype=np.int64),
        2 ** 52 - 1 - rng.integers(0, 2 ** 20, 50_000, dtype=np.int64),  # u near 1: top table cell
        rng.integers(0, 2 ** 12, 10_000, dtype=np.int64),                # u near 2^-52
        np.array([0, 1, 2 ** 51 - 1, 2 ** 51, 2 ** 52 - 1], dtype=np.int64),
    ])
    # cell boundaries of m in [1/2, 1): u = 1/2 + j/2048 (+- one grid step)
    kb = (np.arange(1, 1024, dtype=np.int64) << 41) + (2 ** 51)
    k = np.concatenate([k, kb, kb - 1])
    u = _grid_u(k)
    out = np.empty_like(u)
    fm.fm_neg2_ln(u.ctypes.data, out.ctypes.data, len(u))
    ref = -2 * np.log(u.astype(LD))
    assert np.all(out > 0)
    assert _ulps(out, ref).max() <= 2.0
    # the largest u = 1 - 2^-53: -2 ln u = 2^-52 (1 + 2^-54 ...)
    assert out[np.where(k == 2 ** 52 - 1)[0][0]] == 2.0 ** -52


def test_sqrt(fm):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.random(300_000) * 80, rng.random(1000) * 1e-12, [2.0 ** -52, 1.0, 74.86, 73.47]])
    for f in (fm.fm_sqrt_pos, fm.fm_sqrt_positive):
        out = np.empty_like(x)
        f(x.ctypes.data, out.ctypes.data, len(x))
        assert _ulps(out, np.sqrt(x.astype(LD))).max() <= 1.0


def test_sqrt_pos_zero_is_exact(fm):
    x = np.array([0.0, 2.0 ** -1074, 1e-300])
    out = np.empty_like(x)
    fm.fm_sqrt_pos(x.ctypes.data, out.ctypes.data, len(x))
    assert out[0] == 0.0 and abs(out[2] - 1e-150) < 1e-165


def _t_of_words(w2, w3):
    """t = (i + f)/128 in long double (60 significant bits: exact)."""
    i = (w2 >> 4) & 255
    f = ((w2.astype(np.uint64) >> 12) << 32) | w3.astype(np.uint64)
    return (i.astype(LD) + f.astype(LD) * LD(2.0) ** -52) / 128


def test_sincos_cell(fm):
    rng = np.random.default_rng(2)
    n = 400_000
    w2 = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    w3 = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    # cell edges and centres: f = 0, f = 1/2, f = 1 - 2^-52 in every cell
    cells = np.arange(256, dtype=np.uint32) << 4
    w2 = np.concatenate([w2, cells, cells | 0x80000000, cells | 0xFFFFF000])
    w3 = np.concatenate([w3, np.zeros(256, np.uint32), np.zeros(256, np.uint32),
                         np.full(256, 0xFFFFFFFF, np.uint32)])
    s = np.empty(len(w2))
    c = np.empty(len(w2))
    fm.fm_sincos_cell(w2.ctypes.data, w3.ctypes.data, s.ctypes.data, c.ctypes.data, len(w2))
    ang = PI_LD * _t_of_words(w2, w3)
    # table rounding + three roundings in the angle-addition step: ~2 ulp of 1
    assert np.abs(s - np.sin(ang)).max() < 2.5e-16
    assert np.abs(c - np.cos(ang)).max() < 2.5e-16
    # quarter turns are exact cell edges: t = 0, 1/2, 1, 3/2
    for cell, sv, cv in ((0, 0.0, 1.0), (64, 1.0, 0.0), (128, 0.0, -1.0), (192, -1.0, 0.0)):
        j = len(w2) - 3 * 256 + cell
        assert abs(s[j] - sv) <= 1.2e-16 and abs(c[j] - cv) <= 1.2e-16


def test_normal_pair_matches_oracle(fm):
    """The table-based transform against the oracle's C-library transform of
    the same Philox words."""
    w = OP.blocks(3, 0, 0, 12, 0, 20_000)
    w = np.concatenate([w, np.array([[0, 0, 0, 0], [0xFFFFFFFF, 0xFFFFFFFF, 0, 0],
                                     [0, 0, 0xFFFFFFFF, 0xFFFFFFFF]], dtype=np.uint32)])
    w = np.ascontiguousarray(w, dtype=np.uint32)
    z = np.empty((len(w), 2))
    fm.fm_normal_pair(w.ctypes.data, z.ctypes.data, len(w))
    z0, z1 = OP.box_muller(w)
    # the oracle rounds the angle pi t once (up to 8.9e-16 at t near 2), which
    # the radius r <= 8.6 scales
    tol = 1e-15 * (1.0 + np.hypot(z0, z1))
    assert np.all(np.abs(z[:, 0] - z0) <= tol)
    assert np.all(np.abs(z[:, 1] - z1) <= tol)
