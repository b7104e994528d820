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


@pytest.mark.parametrize("case", list(range(9)))
def test_sparse_pava_is_the_stack_form_bitwise(pv, case):
    v = list(_cases())[case].astype(np.float64)
    ref = OI.pava(v.copy())
    got = np.ascontiguousarray(v.copy())
    pv.pv_pava_sparse(got.ctypes.data_as(ctypes.c_void_p), len(got))
    assert np.array_equal(got, np.asarray(ref)), np.abs(got - ref).max()
