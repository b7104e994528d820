"""Pins for the oracle's noise: Philox4x32-10 words against an independent
library implementation (PyTorch's host Philox engine header), and the
distribution of the Box-Muller normals (Sec. 2.1.3 asks for independent
N(0, dt) increments)."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.stats as st

from oracle import particles as P

_HELPER_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
extern "C" void torch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    uint64_t seed = (uint64_t)key[0] | ((uint64_t)key[1] << 32);
    uint64_t subseq = (uint64_t)ctr[2] | ((uint64_t)ctr[3] << 32);
    uint64_t offset = (uint64_t)ctr[0] | ((uint64_t)ctr[1] << 32);
    at::philox_engine eng(seed, subseq, offset);
    for (int i = 0; i < 4; ++i) out[i] = eng();
}
"""


def _torch_philox_lib():
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) or not shutil.which("g++"):
        pytest.skip("PyTorch Philox header or g++ not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "h.cpp")
    so = os.path.join(d, "h.so")
    with open(src, "w") as f:
        f.write(_HELPER_SRC)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", inc, "-o", so, src])
    L = ctypes.CDLL(so)
    L.torch_philox.argtypes = [ctypes.c_void_p] * 3
    return L


def test_philox_words_match_independent_library(oracle_lib):
    L = _torch_philox_lib()
    rng = np.random.default_rng(1234)
    cases = [np.zeros(4, np.uint32), np.full(4, 0xFFFFFFFF, np.uint32)]
    cases += [rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32) for _ in range(200)]
    keys = [np.zeros(2, np.uint32), np.full(2, 0xFFFFFFFF, np.uint32)]
    keys += [rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32) for _ in range(200)]
    for ctr, key in zip(cases, keys):
        ours = P.philox(ctr, key)
        ref = np.zeros(4, np.uint32)
        L.torch_philox(ctr.ctypes.data, key.ctypes.data, ref.ctypes.data)
        assert np.array_equal(ours, ref), (ctr, key, ours, ref)


def test_block_counter_layout(oracle_lib):
    """or_block is Philox on counter (m, p, tag<<16 | j, instance), key = seed."""
    seed = 0x0123456789ABCDEF
    b = P.blocks(seed, 7, 2, 11, 5, 3, j=4)
    for k in range(3):
        ref = P.philox([11, 5 + k, (2 << 16) | 4, 7], [seed & 0xFFFFFFFF, seed >> 32])
        assert np.array_equal(b[k], ref)


def test_normals_distribution(oracle_lib):
    n = 400_000
    z = P.normals(0, 0, 0, 17, 0, n, 2)
    for col in range(2):
        v = z[:, col]
        assert abs(v.mean()) < 5.0 / np.sqrt(n)
        assert abs(v.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
        ks = st.kstest(v, "norm").statistic
        assert ks < 1.63 / np.sqrt(n)  # KS critical value at alpha = 1e-2
    # the two members of a pair and neighbouring particles are uncorrelated
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5.0 / np.sqrt(n)
    assert abs(np.corrcoef(z[:-1, 0], z[1:, 0])[0, 1]) < 5.0 / np.sqrt(n)


def test_normal_streams_distinct(oracle_lib):
    """Different steps, tags and instances give unrelated numbers."""
    n = 50_000
    a = P.normals(0, 0, 0, 3, 0, n, 1)[:, 0]
    for other in (P.normals(0, 0, 0, 4, 0, n, 1), P.normals(0, 0, 1, 3, 0, n, 1),
                  P.normals(0, 1, 0, 3, 0, n, 1), P.normals(1, 0, 0, 3, 0, n, 1)):
        assert abs(np.corrcoef(a, other[:, 0])[0, 1]) < 5.0 / np.sqrt(n)


def test_normals_extreme_uniforms_are_finite(oracle_lib):
    """u lies in (0, 1), so log(u) is finite for every block."""
    z = P.normals(5, 3, 0, 0, 0, 200_000, 2)
    assert np.all(np.isfinite(z))
    assert np.abs(z).max() < 8.6  # sqrt(-2 log 2^-53) = 8.57 bounds |z|


def test_box_muller_bit_layout_closed_forms(oracle_lib):
    """Words chosen so that u and the angle are known in closed form:
    u = (k + 1/2) 2^-52 from the top 20 bits of w0 and all of w1; the angle
    pi t with t = (i + f)/128, i from bits 4..11 of w2, f from bits 12..31 of
    w2 and all of w3."""
    M = 0xFFFFFFFF
    r_min_u = np.sqrt(106.0 * np.log(2.0))          # u = 2^-53
    cases = [
        # (words, z0, z1)
        ((0, 0, 0, 0), r_min_u, 0.0),
        ((0, 0, 64 << 4, 0), 0.0, r_min_u),             # t = 1/2
        ((0, 0, 128 << 4, 0), -r_min_u, 0.0),           # t = 1
        ((0, 0, 192 << 4, 0), 0.0, -r_min_u),           # t = 3/2
        ((0, 0, 0x80000000, 0), r_min_u * np.cos(np.pi / 256), r_min_u * np.sin(np.pi / 256)),  # f = 1/2
        ((0, 0, 0xF, 0), r_min_u, 0.0),                 # bits 0..3 of w2 are unused
        ((0x800, 0, 0, 0), r_min_u, 0.0),               # bits 0..11 of w0 are unused
    ]
    for w, e0, e1 in cases:
        z0, z1 = P.box_muller(np.array(w, dtype=np.uint32))
        assert abs(z0[0] - e0) < 4e-15 and abs(z1[0] - e1) < 4e-15, (w, z0, z1, e0, e1)
    # u = 1 - 2^-53 (largest): radius sqrt(-2 ln(1 - 2^-53)) = 2^-26 (1 + O(2^-53))
    z0, _ = P.box_muller(np.array((M, M, 0, 0), dtype=np.uint32))
    assert abs(z0[0] / 2.0 ** -26 - 1.0) < 1e-12
    # u = 1/2 + 2^-53 (k = 2^51): radius sqrt(2 ln 2) to first order
    z0, _ = P.box_muller(np.array((0x80000000, 0, 0, 0), dtype=np.uint32))
    assert abs(z0[0] - np.sqrt(2.0 * np.log(2.0))) < 1e-15
    # w1 is the low word of k: k = 1 gives u = 3 * 2^-53
    z0, _ = P.box_muller(np.array((0, 1, 0, 0), dtype=np.uint32))
    assert abs(z0[0] - np.sqrt(-2.0 * np.log(3.0 * 2.0 ** -53))) < 1e-14
    # w3 is the low word of f: f = 2^-52 moves the angle by pi 2^-59
    _, z1 = P.box_muller(np.array((0, 0, 0, 1), dtype=np.uint32))
    assert abs(z1[0] - r_min_u * np.pi * 2.0 ** -59) < 1e-30


def test_box_muller_angle_cells_uniform(oracle_lib):
    """The 256 angle cells (bits 4..11 of w2) are equally likely and the
    radius is independent of the cell (chi-square, alpha = 1e-3)."""
    n = 256_000
    b = P.blocks(9, 0, 0, 5, 0, n)
    cell = (b[:, 2] >> 4) & 255
    cnt = np.bincount(cell, minlength=256)
    assert st.chisquare(cnt).pvalue > 1e-3
    z = P.normals(9, 0, 0, 5, 0, n, 2)
    ang = np.mod(np.arctan2(z[:, 1], z[:, 0]), 2 * np.pi)
    # the angle sits inside its cell [i, i+1) pi/128
    inside = (ang >= cell * np.pi / 128 - 1e-12) & (ang < (cell + 1) * np.pi / 128 + 1e-12)
    assert inside.all()
    r2 = z[:, 0] ** 2 + z[:, 1] ** 2
    # -2 ln u is Exp(1/2): chi-square with 2 degrees of freedom, independent of the cell
    assert st.kstest(r2, "chi2", args=(2,)).pvalue > 1e-3
    assert abs(np.corrcoef(r2, cell)[0, 1]) < 5.0 / np.sqrt(n)


def test_box_muller_f32_bit_layout_closed_forms(oracle_lib):
    """Normals of the single-precision propagator: u = (k + 1/2) 2^-24 from the
    top 24 bits of w0, the angle pi t with t = (i + f)/128, i from bits 4..11
    of w2 and f from bits 12..31 of w2 (20 bits); w1, w3 and the low bits of
    w0 and w2 take no part."""
    M = 0xFFFFFFFF
    r_min_u = np.sqrt(50.0 * np.log(2.0))           # u = 2^-25
    cases = [
        ((0, 0, 0, 0), r_min_u, 0.0),
        ((0, 0, 64 << 4, 0), 0.0, r_min_u),             # t = 1/2
        ((0, 0, 128 << 4, 0), -r_min_u, 0.0),           # t = 1
        ((0, 0, 192 << 4, 0), 0.0, -r_min_u),           # t = 3/2
        ((0, 0, 0x80000000, 0), r_min_u * np.cos(np.pi / 256), r_min_u * np.sin(np.pi / 256)),  # f = 1/2
        ((0, 0, 0xF, 0), r_min_u, 0.0),                 # bits 0..3 of w2 are unused
        ((0xFF, 0, 0, 0), r_min_u, 0.0),                # bits 0..7 of w0 are unused
        ((0, M, 0, M), r_min_u, 0.0),                   # w1 and w3 are unused
    ]
    for w, e0, e1 in cases:
        z0, z1 = P.box_muller_f32(np.array(w, dtype=np.uint32))
        assert abs(z0[0] - e0) < 4e-15 and abs(z1[0] - e1) < 4e-15, (w, z0, z1, e0, e1)
    # u = 1 - 2^-25 (largest): radius sqrt(-2 ln(1 - 2^-25)) = 2^-12 (1 + 2^-27 + ...)
    z0, _ = P.box_muller_f32(np.array((M, 0, 0, 0), dtype=np.uint32))
    assert abs(z0[0] / 2.0 ** -12 - 1.0) < 1e-8
    # k = 1 (bit 8 of w0): u = 3 * 2^-25
    z0, _ = P.box_muller_f32(np.array((0x100, 0, 0, 0), dtype=np.uint32))
    assert abs(z0[0] - np.sqrt(-2.0 * np.log(3.0 * 2.0 ** -25))) < 1e-14
    # bit 12 of w2 is the lowest bit of f: f = 2^-20 moves the angle by pi 2^-27
    _, z1 = P.box_muller_f32(np.array((0, 0, 1 << 12, 0), dtype=np.uint32))
    assert abs(z1[0] - r_min_u * np.sin(np.pi * 2.0 ** -27)) < 1e-22


def test_box_muller_f32_is_the_double_transform_of_its_bits(oracle_lib):
    """The single-precision normals are the double-precision transform of a
    block that carries the same bits: with w1 = (bits 8..11 of w0) 2^28 +
    2^27 and w3 = 0, the double transform's u is the single one's plus
    2^-53 and its angle is the same, so the pairs agree to
    2^-53 / (u r) <= 2^-28 / 5.89 < 1e-9 (u >= 2^-25)."""
    rng = np.random.default_rng(77)
    w = rng.integers(0, 2 ** 32, (4000, 4), dtype=np.uint64).astype(np.uint32)
    w[:3, 0] = [0, 0xFFFFFFFF, 0x80000000]
    a0, a1 = P.box_muller_f32(w)
    wd = w.copy()
    wd[:, 1] = (((w[:, 0] >> 8) & 0xF) << 28) | (1 << 27)
    wd[:, 3] = 0
    b0, b1 = P.box_muller(wd)
    assert np.abs(a0 - b0).max() < 1e-9 and np.abs(a1 - b1).max() < 1e-9
    # and differs from the full-width pair of the original words (the bits
    # below the top 24 of u matter there)
    c0, _ = P.box_muller(w)
    assert np.abs(a0 - c0).max() > 1e-7


def test_box_muller_f32_distribution(oracle_lib):
    n = 200_000
    b = P.blocks(4, 0, 0, 9, 0, n)
    z0, z1 = P.box_muller_f32(b)
    for v in (z0, z1):
        assert abs(v.mean()) < 5.0 / np.sqrt(n)
        assert abs(v.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
        assert st.kstest(v, "norm").statistic < 1.63 / np.sqrt(n)
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 5.0 / np.sqrt(n)
    assert np.abs(np.hypot(z0, z1)).max() <= np.sqrt(50.0 * np.log(2.0)) + 1e-12


def test_coupling_and_instance_params(oracle_lib):
    a = P.coupling(0, 0, 32)
    assert a.shape == (32,) and np.all(a >= 0.5) and np.all(a < 1.5)
    assert len(set(a.tolist())) == 32
    seen_n, seen_k = set(), set()
    for inst in range(256):
        eps, lam, n, k = P.instance_params(0, inst)
        assert 1e-3 <= eps <= 1e-1 and 0.5 <= lam <= 2.0
        assert n in [2 ** e for e in range(12, 19)] and 8 <= k <= 64
        seen_n.add(n)
        seen_k.add(k)
    assert len(seen_n) == 7 and len(seen_k) > 40


def test_instance_params_distributions(oracle_lib):
    """The batched workload's draws over 4096 instances follow their laws:
    log10 eps ~ U(-3, -1), lambda ~ U(0.5, 2) (Kolmogorov-Smirnov at the
    0.1 % level), log2 P uniform on 12..18 and the slice count uniform on
    8..64 (chi-square at the 0.1 % level), the four independent of each
    other (rank correlations).  A slip in a range (10^(-3+u), 0.5 + u/2)
    or in an integer draw (floor(6u), 8 + floor(56u)) fails one of them."""
    n = 4096
    d = np.array([P.instance_params(0, i) for i in range(n)], dtype=np.float64)
    le, lam, lg, k = np.log10(d[:, 0]), d[:, 1], np.log2(d[:, 2]), d[:, 3]
    assert st.kstest(le, st.uniform(loc=-3.0, scale=2.0).cdf).pvalue > 1e-3
    assert st.kstest(lam, st.uniform(loc=0.5, scale=1.5).cdf).pvalue > 1e-3
    assert le.min() > -3.0 and le.max() < -1.0 and lam.min() > 0.5 and lam.max() < 2.0
    assert np.array_equal(lg, np.round(lg))
    cnt = np.array([(lg == e).sum() for e in range(12, 19)])
    assert cnt.sum() == n and st.chisquare(cnt).pvalue > 1e-3
    cnt = np.array([(k == v).sum() for v in range(8, 65)])
    assert cnt.sum() == n and st.chisquare(cnt).pvalue > 1e-3
    cols = [le, lam, lg, k]
    for a in range(4):
        for b in range(a + 1, 4):
            assert abs(st.spearmanr(cols[a], cols[b]).statistic) < 5.0 / np.sqrt(n)


def test_coupling_distribution(oracle_lib):
    """a_i ~ U(0.5, 1.5) over 4096 coefficients (Kolmogorov-Smirnov at the
    0.1 % level; a slip to 0.5 + u/2 or to 1 + u fails it), and the
    coefficients of one seed do not depend on how many are drawn."""
    a = P.coupling(0, 0, 4096)
    assert st.kstest(a, st.uniform(loc=0.5, scale=1.0).cdf).pvalue > 1e-3
    assert a.min() >= 0.5 and a.max() < 1.5
    assert np.array_equal(P.coupling(0, 0, 32), a[:32])
    b = P.coupling(1, 0, 4096)
    assert abs(st.spearmanr(a, b).statistic) < 5.0 / np.sqrt(4096)
