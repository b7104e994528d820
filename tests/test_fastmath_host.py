"""The FP64 helpers of the Box-Muller transform (log on (0, 1], sqrt, and
sin/cos of pi t on [0, 2]) against the C library, on the host build of
the same source (the device build swaps only the reciprocal seeds)."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1912_09240_amd", "csrc")


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
    for f in (L.fm_log_unit, L.fm_sqrt_pos):
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
    L.fm_sincos_half_turn.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_long]
    return L


def _ulps(a, ref):
    return np.abs(a - ref) / np.spacing(np.abs(ref))


def test_log_unit(fm):
    rng = np.random.default_rng(0)
    u = np.concatenate([rng.random(500_000), 1 - rng.random(100_000) * 1e-6, [1.0, 0.5, 2.0 ** -54, 0.7071067811865476,
                        np.nextafter(0.7071067811865476, 0), 0.75, 1 - 2 ** -53]])
    u = u[u > 0]
    out = np.empty_like(u)
    fm.fm_log_unit(u.ctypes.data, out.ctypes.data, len(u))
    ref = np.log(u)
    nz = ref != 0
    assert np.all(out[~nz] == 0.0)
    assert _ulps(out[nz], ref[nz]).max() <= 4


def test_sqrt_pos(fm):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.random(300_000) * 80, rng.random(1000) * 1e-12, [0.0, 1.0, 74.86]])
    out = np.empty_like(x)
    fm.fm_sqrt_pos(x.ctypes.data, out.ctypes.data, len(x))
    assert out[x == 0].max() == 0.0
    assert _ulps(out[x > 0], np.sqrt(x[x > 0])).max() <= 1


def test_sincos_half_turn(fm):
    rng = np.random.default_rng(2)
    t = np.concatenate([rng.random(500_000) * 2, np.arange(0, 2.001, 0.0625), [np.nextafter(2, 0), 0.5, 1.5]])
    s = np.empty_like(t)
    c = np.empty_like(t)
    fm.fm_sincos_half_turn(t.ctypes.data, s.ctypes.data, c.ctypes.data, len(t))
    ang = t * np.pi  # reference angle rounded once; its rounding bounds the comparison
    assert np.abs(s - np.sin(ang)).max() < 4e-16 * 4
    assert np.abs(c - np.cos(ang)).max() < 4e-16 * 4
    # exact half-turn and quarter-turn points
    for tv, sv, cv in ((0.0, 0.0, 1.0), (0.5, 1.0, 0.0), (1.0, 0.0, -1.0), (1.5, -1.0, 0.0), (2.0, 0.0, 1.0)):
        i = np.where(t == tv)[0][0]
        assert abs(s[i] - sv) <= 2.3e-16 and abs(c[i] - cv) <= 2.3e-16
    assert np.abs(s * s + c * c - 1).max() < 1e-15


def test_sqrt_pos_zero_is_exact(fm):
    x = np.array([0.0, 2.0 ** -1074, 1e-300])
    out = np.empty_like(x)
    fm.fm_sqrt_pos(x.ctypes.data, out.ctypes.data, len(x))
    assert out[0] == 0.0 and abs(out[2] - 1e-150) < 1e-165
