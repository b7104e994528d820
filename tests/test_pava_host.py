"""The library's sparse pool-adjacent-violators pass (host build of the same
source the quantile iterators inline) against the oracle's stack form, bit
for bit, on inputs with many violations, exact ties, long decreasing runs
and none at all."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import iterate as OI

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def pv():
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    so = os.path.join(d, "pv.so")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                           "-I", os.path.join(ROOT, "paper_1912_09240_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "pava_host.hip"), "-o", so], stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(so)
    L.pv_pava_sparse.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.pv_pava_sparse.restype = ctypes.c_int
    L.pv_pava_stretches.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.pv_pava_stretches.restype = ctypes.c_int
    L.pv_mean_above.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int, ctypes.c_void_p]
    L.pv_mean_above.restype = None
    return L


def _cases():
    rng = np.random.default_rng(17)
    yield np.sort(rng.random(50))                       # monotone: identity
    yield rng.random(200)                               # violations everywhere
    yield np.round(rng.random(300) * 8) / 8             # exact ties
    yield np.linspace(1.0, 0.0, 101)                    # one decreasing run
    yield np.concatenate([np.linspace(0, 1, 40), np.linspace(0.9, 0.1, 30), np.linspace(0.2, 3, 60)])
    yield np.cumsum(rng.normal(0.01, 0.02, 3000))      # a noisy rising quantile function
    x = np.cumsum(rng.random(1000) * 1e-3)
    x[::37] -= 5e-3                                     # isolated dips
    yield x
    yield np.array([1.0, 1.0, 0.0, 2.0, 1.5, 1.5, 1.5, 0.5, 4.0])
    yield np.array([3.0])
    # zig-zag runs: violations every other position, as where the levels of
    # three cdfs interleave
    z = np.cumsum(rng.random(2000) * 1e-3)
    z[1::2] -= 2e-3 * rng.random(1000)
    yield z
    w = np.cumsum(rng.random(3000))
    for c0 in (200, 900, 1500, 2600):
        w[c0:c0 + 60:2] += 3.0
    yield w
    # near ties: runs of one value moved by a few units in the last place,
    # so that neighbouring pool means differ only in their rounding
    base = np.repeat(np.round(rng.random(80), 2), 6)
    yield base + rng.integers(-3, 4, base.size) * np.spacing(base)
    # pools of many thirds and tenths, whose sums round
    t = np.repeat(np.arange(1, 40) / 3.0, 7)[::-1].copy()
    t[::5] += 0.1
    yield t


@pytest.mark.parametrize("case", list(range(13)))
def test_sparse_pava_is_the_stack_form_bitwise(pv, case):
    v = list(_cases())[case].astype(np.float64)
    ref = OI.pava(v.copy())
    got = np.ascontiguousarray(v.copy())
    pv.pv_pava_sparse(got.ctypes.data_as(ctypes.c_void_p), len(got))
    assert np.array_equal(got, np.asarray(ref)), np.abs(got - ref).max()


@pytest.mark.parametrize("case", list(range(13)))
def test_stretch_decomposition_is_the_stack_form_bitwise(pv, case):
    """The stretches of the block pass, each on its own, with the cuts that
    the serial pass would cross dropped: the stack form's result bit for bit."""
    v = list(_cases())[case].astype(np.float64)
    ref = np.asarray(OI.pava(v.copy()))
    got = np.ascontiguousarray(v.copy())
    pv.pv_pava_stretches(got.ctypes.data_as(ctypes.c_void_p), len(got))
    assert np.array_equal(got, ref), np.abs(got - ref).max()


def test_stretch_decomposition_on_random_walks(pv):
    rng = np.random.default_rng(5)
    rounds = []
    for t in range(300):
        n = int(rng.integers(2, 400))
        v = np.cumsum(rng.normal(rng.random() * 0.1, 1.0, n))
        if t % 3 == 0:
            v = np.round(v)  # ties
        ref = np.asarray(OI.pava(v.copy()))
        got = np.ascontiguousarray(v.copy())
        rounds.append(pv.pv_pava_stretches(got.ctypes.data_as(ctypes.c_void_p), n))
        assert np.array_equal(got, ref), (t, np.abs(got - ref).max())
    assert max(rounds) >= 1


def test_mean_comparison_is_that_of_the_rounded_quotients(pv):
    """The library decides S/C > S'/C' from cross products where they are
    far apart and from the quotients otherwise: on near ties (means equal in
    exact arithmetic, or a few units in the last place apart), wide
    magnitudes, zeros, infinities and NaN it answers as the comparison of
    the two rounded quotients does."""
    rng = np.random.default_rng(23)
    n = 200_000
    ca = rng.integers(1, 65536, n).astype(np.int32)
    cb = rng.integers(1, 65536, n).astype(np.int32)
    mean = rng.normal(0.0, 1.0, n) * 10.0 ** rng.integers(-300, 300, n)
    kind = rng.integers(0, 4, n)
    with np.errstate(over="ignore"):
        a = mean * ca
        near = (mean + rng.integers(-4, 5, n) * np.spacing(mean)) * cb
        b = np.where(kind == 0, mean * cb,                  # ties in exact arithmetic
                     np.where(kind == 1, near, np.where(kind == 2, rng.normal(0.0, 1.0, n) * cb, -a * cb / ca)))
    a[:8] = [0.0, -0.0, np.inf, -np.inf, np.nan, 1.0, 5e-324, -5e-324]
    b[:8] = [-0.0, 0.0, np.inf, 1.0, 1.0, np.nan, 0.0, 5e-324]
    out = np.zeros(n, dtype=np.int32)
    p = lambda z: np.ascontiguousarray(z).ctypes.data_as(ctypes.c_void_p)
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    pv.pv_mean_above(p(a), p(ca), p(b), p(cb), n, p(out))
    with np.errstate(invalid="ignore", over="ignore"):
        ref = (a / ca.astype(np.float64)) > (b / cb.astype(np.float64))
    assert np.array_equal(out.astype(bool), ref)
    # the near ties do reach the quotients: their rounded means are equal or
    # a few units apart, both outcomes occurring
    close = (kind == 1) | (kind == 0)
    assert ref[close].any() and (~ref[close]).any()
