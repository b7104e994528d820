"""The C-ABI library builds, loads and exports every entry point declared in
include/pr.h; argument validation rejects bad calls before touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_1912_09240_amd as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not pr.available():
        from paper_1912_09240_amd import build
        build.build()
    return pr.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in pr.__all__, n


def test_version_and_error_string(lib):
    assert pr.pr_version() == 1
    assert isinstance(pr.pr_last_error(), str)


def test_workspace_size_is_monotone(lib):
    a = pr.pr_restrict_workspace_size(1000, 3)
    b = pr.pr_restrict_workspace_size(100000, 3)
    c = pr.pr_restrict_workspace_size(100000, 3, pr.PR_F32)
    assert 0 < a < b and c < b
    # keys (2 x 8 B) + payload (2 x 4 B) per element at least
    assert b >= 100000 * 3 * 24


def test_validation_rejects_before_launch(lib):
    L = lib
    # NULL sde
    assert L.pr_init_ensemble(None, 0, 0, 10, None, None, None) == -1
    assert "sde" in pr.pr_last_error()
    # bad precision / d
    bad = pr.Sde(d=5).c()
    assert L.pr_init_ensemble(ctypes.byref(bad), 0, 0, 10, None, None, None) == -1
    bad = pr.Sde(precision=16).c()
    assert L.pr_init_ensemble(ctypes.byref(bad), 0, 0, 10, None, None, None) == -1
    # negative eps
    bad = pr.Sde(eps=-1.0).c()
    assert L.pr_init_ensemble(ctypes.byref(bad), 0, 0, 10, None, None, None) == -1
    # slices outside the schedule
    s, c = pr.Sde().c(), pr.Schedule(100, 4, 1e-3).c()
    assert L.pr_fine_propagate(ctypes.byref(s), ctypes.byref(c), 0, 0, 10, 3, 2, None, None, None) == -1
    # schedule with fewer steps than slices
    c2 = pr.Schedule(3, 4, 1e-3).c()
    assert L.pr_fine_propagate(ctypes.byref(s), ctypes.byref(c2), 0, 0, 10, 0, 1, None, None, None) == -1
    # workspace too small
    assert L.pr_restrict_quantiles(ctypes.c_void_p(16), 64, 1000, 2, 100, None, ctypes.c_void_p(16), None, None,
                                   None, None, None, ctypes.c_void_p(16), 10, None) == -3
    # grid checks
    g = pr.Grid(n_cells=2).c()
    h = ctypes.c_void_p()
    assert L.pr_coarse_create(ctypes.byref(s), ctypes.byref(pr.Schedule(100, 4, 1e-3).c()), ctypes.byref(g), None,
                              ctypes.byref(h)) == -1
    g = pr.Grid(x_lo=1.0, x_hi=0.0).c()
    assert L.pr_parareal_create(ctypes.byref(s), ctypes.byref(pr.Schedule(100, 4, 1e-3).c()), ctypes.byref(g), 0,
                                0, 10, 0, None, ctypes.byref(h)) == -1
    # unknown flags
    g = pr.Grid().c()
    assert L.pr_parareal_create(ctypes.byref(s), ctypes.byref(pr.Schedule(100, 4, 1e-3).c()), ctypes.byref(g), 0,
                                0, 10, 64, None, ctypes.byref(h)) == -1
    # matching without pointers
    assert L.pr_match_quantiles(None, None, None, 10, 1, 100, None, None, 64, None) == -1
    # knots of matched ensembles: pointers, precision, sizes and the workspace
    # are checked before any launch
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.pr_match_knots(None, p, 10, 1, 100, 64, p, 1 << 20, p, p, None) == -1
    assert L.pr_match_knots(p, p, 10, 1, 100, 16, p, 1 << 20, p, p, None) == -1
    assert L.pr_match_knots(p, p, 0, 1, 100, 64, p, 1 << 20, p, p, None) == -1
    assert L.pr_match_knots(p, p, 10, 0, 100, 64, p, 1 << 20, p, p, None) == -1
    assert L.pr_match_knots(p, p, 10, 1, 0, 64, p, 1 << 20, p, p, None) == -1
    assert L.pr_match_knots(p, p, 1 << 20, 4, 100, 64, p, 1024, p, p, None) == -3
    assert L.pr_parareal_knot_sorts(None) == -1
    assert L.pr_parareal_batch_knot_sorts(None, None) == -1
    assert L.pr_parareal_batch_info(None, None, None, None, None, None) == -1
    assert L.pr_quantile_jump(p, p, p, -1, 100, p, None) == -1
    assert L.pr_quantile_jump(p, p, p, 3, 0, p, None) == -1
    assert L.pr_quantile_jump(p, p, p, 3, 2048, p, None) == -1
    assert L.pr_quantile_jump(None, p, p, 3, 100, p, None) == -1
    assert L.pr_quantile_jump(None, None, None, 0, 100, None, None) == 0
    # the restriction without allocation: arguments and the size of the
    # static scratch are checked before the device is touched
    assert L.pr_restrict_quantiles_static(None, 64, 1000, 2, 100, None, p, None, None, None, None, None, None) == -1
    assert L.pr_restrict_quantiles_static(p, 64, 1000, 2, 100, None, None, None, None, None, None, None, None) == -1
    assert L.pr_restrict_quantiles_static(p, 16, 1000, 2, 100, None, p, None, None, None, None, None, None) == -1
    assert L.pr_restrict_quantiles_static(p, 64, 1 << 20, 3, 100, None, p, None, None, None, None, None, None) == -3
    assert "static scratch" in pr.pr_last_error()
    # iterate on a NULL handle
    assert L.pr_parareal_iterate(None, 1, None, None, None) == -1


def test_chem_validation_and_host_mean(lib):
    """The chemical system's arguments are checked before any launch, and the
    fast-variable mean (host code) agrees with the oracle's trapezoidal rule."""
    from oracle import chem as OCH
    L = lib
    s = pr.Schedule(100, 4, 1e-3).c()
    assert L.pr_chem_init_ensemble(None, 0, 0, 10, None, None, None) == -1
    for bad in (pr.Chem(k=(60.0, 1.0, 4.8e-3, 0.666e-5, 0.833, 0.0)), pr.Chem(eps=-1.0),
                pr.Chem(k=(60.0, -1.0, 4.8e-3, 0.666e-5, 0.833, 1.0)), pr.Chem(x0=(0.0, 1.0))):
        c = bad.c()
        assert L.pr_chem_fine_propagate(ctypes.byref(c), ctypes.byref(s), 0, 0, 10, 0, 1, None, None, None) == -1
    c = pr.Chem().c()
    assert L.pr_chem_fine_propagate(ctypes.byref(c), ctypes.byref(s), 0, 0, 10, 3, 2, None, None, None) == -1
    h = ctypes.c_void_p()
    g = pr.Grid(n_cells=2000, x_lo=0.0, x_hi=600.0).c()
    assert L.pr_parareal_hist_create_chem(ctypes.byref(c), ctypes.byref(s), ctypes.byref(g), 0, 0, 10, 0, 0, 0, None,
                                          ctypes.byref(h)) == -1
    g = pr.Grid(n_cells=600, x_lo=-400.0, x_hi=600.0).c()  # Dbar < 0 at the left end
    assert L.pr_chem_coarse_create(ctypes.byref(c), ctypes.byref(s), ctypes.byref(g), None, ctypes.byref(h)) == -1
    for k in (OCH.K_DEFAULT, (60.0, 1.0, 0.0, 0.0, 0.833, 1.0), (30.0, 0.5, 2e-3, 1e-6, 1.0, 0.5)):
        got = pr.pr_chem_mean_fast(pr.Chem(k=k))
        ref = OCH.mean_fast(OCH.Chem(k=k))
        assert abs(got - ref) < 1e-12 * abs(ref), (k, got, ref)
    # E(y) <= 0 somewhere on [0, 1000] is an error, not a NaN
    with pytest.raises(pr.PrError):
        pr.pr_chem_mean_fast(pr.Chem(k=(0.0, 0.0, 4.8e-3, 0.0, 0.833, 1.0)))


def test_advection_validation(lib):
    L = lib
    s, g = pr.Schedule(100, 4, 1e-2).c(), pr.Grid(n_cells=100, x_lo=-8.0, x_hi=8.0).c()
    h = ctypes.c_void_p()
    assert L.pr_advection_coarse_create(0.0, 1.0, ctypes.byref(s), ctypes.byref(g), None, ctypes.byref(h)) == -1
    assert L.pr_advection_coarse_create(1.0, -1.0, ctypes.byref(s), ctypes.byref(g), None, ctypes.byref(h)) == -1
    assert L.pr_parareal_fp_create(None, None, ctypes.byref(g), None, 0, 0, None, ctypes.byref(h)) == -1
    assert L.pr_parareal_fp_iterate(None, 1, None, None, None) == -1
    assert L.pr_parareal_fp_iteration(None) == -1
