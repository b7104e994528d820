"""GPU parity of the chemical-reaction workload (Sec. 2.1.2, Sec. 2.2.1,
Sec. 2.2.2) through the C ABI against the oracle on the same seeded inputs:
the lognormal initial ensemble, the multiplicative-noise fine propagator (all
slices in one launch; at the full workload on sampled particles), the
coarse exponentials, and the histogram-state driver on this model."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import chem as OCH
from oracle import coarse as OC
from oracle import histogram as H
from oracle import iterate as OI

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert pr.available(), "libpr.so not built"
    return torch


def _copy_device(ptr, count):
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    out = np.empty(count, dtype=np.float64)
    rc = hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr), ctypes.c_size_t(count * 8),
                       ctypes.c_int(2))
    assert rc == 0
    return out


@pytest.mark.parametrize("n", [1, 10_007])
def test_chem_initial_ensemble(torch_dev, n):
    torch = torch_dev
    _say(f"chem init n={n}")
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_chem_init_ensemble(pr.Chem(), 3, 1, n, x, y)
    xo, yo = OCH.init_ensemble(OCH.Chem(), 3, 1, n)
    assert np.abs(x.cpu().numpy() - xo).max() < 1e-13 * xo.max()
    assert np.abs(y.cpu().numpy() - yo[0]).max() < 1e-13 * yo.max()


@pytest.mark.parametrize("n,S,K,dt,eps", [(4_099, 3_000, 3, 1e-3, 2.5e-2), (513, 800, 5, 1e-3, 2.5e-3),
                                          (1_000, 400, 2, 1e-2, 0.1)])
def test_chem_fine_all_slices(torch_dev, n, S, K, dt, eps):
    """All K slices in one launch, each from its own start state, against the
    oracle slice by slice (includes y = 0 and states below it where D and E
    are clipped to 0)."""
    torch = torch_dev
    _say(f"chem fine n={n} S={S} K={K} dt={dt} eps={eps}")
    oc = OCH.Chem(eps=eps)
    x0, y0 = OCH.init_ensemble(oc, 5, 0, n)
    xs = np.stack([x0 * (1.0 + 0.3 * k) for k in range(K)])
    ys = np.stack([y0[0] * (1.0 + 0.7 * k) for k in range(K)])
    # y = 0, and states far below it where E(y) < 0 and D < 0 are clipped to 0
    ys[0, :4] = [0.0, -200.0, -300.0, 1.5]
    xs[0, :4] = [50.0, 20.0, -10.0, 100.0]
    x = torch.from_numpy(xs.copy()).cuda()
    y = torch.from_numpy(ys.copy()).cuda()
    pr.pr_chem_fine_propagate(pr.Chem(eps=eps), pr.Schedule(S, K, dt), 5, 0, n, 0, K, x, y)
    xg, yg = x.cpu().numpy(), y.cpu().numpy()
    b = OI.slice_bounds(S, K)
    for k in range(K):
        xr, yr = OCH.em_propagate(oc, 5, 0, xs[k], ys[k], b[k], b[k + 1], dt)
        assert np.abs(xg[k] - xr).max() < 1e-11 * max(1.0, np.abs(xr).max()), k
        assert np.abs(yg[k] - yr[0]).max() < 1e-11 * max(1.0, np.abs(yr).max()), k


def test_chem_fine_full_workload_sampled(torch_dev):
    """Table 1 workload (P = 1e5, N = 20, T = 40, dt = 1e-3): one launch over
    all slices, compared with the oracle on 64 particles of every slice
    (a run of particles across the last partial tile included)."""
    torch = torch_dev
    n, K, S, dt = 100_000, 20, 40_000, 1e-3
    _say(f"chem fine full n={n} K={K} S={S}")
    oc = OCH.Chem()
    x0, y0 = OCH.init_ensemble(oc, 9, 0, n)
    xs = np.stack([x0 + 5.0 * k for k in range(K)])
    ys = np.stack([y0[0] + 12.0 * k for k in range(K)])
    x = torch.from_numpy(xs.copy()).cuda()
    y = torch.from_numpy(ys.copy()).cuda()
    pr.pr_chem_fine_propagate(pr.Chem(), pr.Schedule(S, K, dt), 9, 0, n, 0, K, x, y)
    xg, yg = x.cpu().numpy(), y.cpu().numpy()
    assert np.isfinite(xg).all() and np.isfinite(yg).all()
    b = OI.slice_bounds(S, K)
    for k in range(K):
        p0 = (k * 4_999) % (n - 64) if k < K - 1 else n - 64
        xr, yr = OCH.em_propagate(oc, 9, 0, xs[k, p0:p0 + 64], ys[k, p0:p0 + 64], b[k], b[k + 1], dt, p0=p0)
        assert np.abs(xg[k, p0:p0 + 64] - xr).max() < 1e-10 * np.abs(xr).max(), k
        assert np.abs(yg[k, p0:p0 + 64] - yr[0]).max() < 1e-10 * np.abs(yr).max(), k


@pytest.mark.parametrize("I,S,K,dt", [(600, 40_000, 20, 1e-3), (150, 3_000, 7, 1e-3)])
def test_chem_coarse_matches_oracle(torch_dev, I, S, K, dt):
    torch = torch_dev
    _say(f"chem coarse I={I} K={K}")
    h = pr.pr_chem_coarse_create(pr.Chem(), pr.Schedule(S, K, dt), pr.Grid(n_cells=I, x_lo=0.0, x_hi=600.0))
    try:
        torch.cuda.synchronize()
        prop = OCH.Propagator(OC.Grid(I, 0.0, 600.0), OCH.Chem())
        b = OI.slice_bounds(S, K)
        for s in (0, K - 1):
            Eg = _copy_device(pr.pr_coarse_matrix(h, s), I * I).reshape(I, I)
            Eo = prop.expm((b[s + 1] - b[s]) * dt)
            assert np.abs(Eg - Eo).max() < 1e-11, s
            assert np.abs(Eg.sum(0) - 1).max() < 1e-11, s
    finally:
        pr.pr_coarse_destroy(h)


@pytest.mark.parametrize("it,mt", [(pr.PR_J_ADD, pr.PR_M_RESAMPLE), (pr.PR_J_MULT, pr.PR_M_REWEIGHT),
                                   (pr.PR_J_ROT, pr.PR_M_MARGINAL), (pr.PR_J_QUANTILE, pr.PR_M_RESAMPLE_DET),
                                   (pr.PR_J_QUANTILE, pr.PR_M_MARGINAL)])
def test_chem_hist_driver_matches_oracle(torch_dev, it, mt):
    """The histogram-state driver on the chemical model against the oracle,
    state by state over two iterations, within 1e-8 (particles) and 1e-12
    (masses) plus 100 times what the oracle itself moves when its coarse
    products are summed in the other order.  Cells of 10 (60 on
    [0, 600]): on much coarser cells the generator's coefficients span many
    orders of magnitude across one cell and the exponential itself is
    ill-conditioned (two correct routes to it differ by 1e-9 at 20 cells)."""
    torch = torch_dev
    _say(f"chem hist driver it={it} mt={mt}")
    n, K, T, dt, I = 2000, 3, 3.0, 1e-2, 60
    S = int(round(T / dt))
    g, og = pr.Grid(n_cells=I, x_lo=0.0, x_hi=600.0), OC.Grid(I, 0.0, 600.0)
    h = pr.pr_parareal_hist_create_chem(pr.Chem(), pr.Schedule(S, K, T / S), g, 4, 0, n, it, mt)
    orc, hp = H.micmac_parareal_hist(OCH.Chem(), 4, 0, n, T, dt, K, og, it, mt)
    # the same oracle with its coarse products summed in reverse order: how
    # far a 1e-16 change of the coarse results moves the states (the
    # union-of-levels quantile iterator divides by differences of nearly
    # equal levels where the fine histograms have empty interior cells)
    alt, _ = H.micmac_parareal_hist(OCH.Chem(), 4, 0, n, T, dt, K, og, it, mt)
    alt.coarse = lambda m, r: np.maximum(hp["E"][m][:, ::-1] @ r[::-1], 0.0)
    try:
        for k in range(3):
            if k > 0:
                pr.pr_parareal_hist_iterate(h, 1)
                orc.iterate()
                alt.iterate()
            for t in range(K + 1):
                x = torch.empty(n, dtype=torch.float64, device="cuda")
                w = torch.empty(n, dtype=torch.float64, device="cuda")
                rho = torch.empty(I, dtype=torch.float64, device="cuda")
                pr.pr_parareal_hist_state(h, t, x=x, w=w, rho=rho)
                u = orc.u[t]
                x_tol = 1e-8 + 100.0 * np.abs(alt.u[t].x - u.x).max()
                rho_tol = 1e-12 + 100.0 * np.abs(alt.rho[t] - orc.rho[t]).max()
                assert np.abs(x.cpu().numpy() - u.x).max() < x_tol, (k, t)
                assert np.abs(w.cpu().numpy() - u.w).max() < 1e-14, (k, t)
                assert np.abs(rho.cpu().numpy() - orc.rho[t]).max() < rho_tol, (k, t)
    finally:
        pr.pr_parareal_hist_destroy(h)


def test_chem_hist_driver_full_workload(torch_dev):
    """Table 1 workload (P = 1e5, N = 20, T = 40, grid [0, 600] with h = 1):
    after one iteration of the additive iterator with stratified resampling
    the state at t_1 is the fine propagation of X0 bitwise (Sec. 3.3.3), the
    histograms are probability vectors, and the error to a serial run of the
    library's own kernels is zero at t_1."""
    torch = torch_dev
    n, K, S, dt, I = 100_000, 20, 40_000, 1e-3, 600
    _say(f"chem hist full n={n} K={K} S={S} I={I}")
    chem, sched, g = pr.Chem(), pr.Schedule(S, K, dt), pr.Grid(n_cells=I, x_lo=0.0, x_hi=600.0)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_chem_init_ensemble(chem, 2, 0, n, x, y)
    ref = torch.empty((K + 1, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_workspace_size(1, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_restrict(x, None, n, 1, g, ref[0], ws)
    xs = [x.clone()]
    for s_ in range(K):
        pr.pr_chem_fine_propagate(chem, sched, 2, 0, n, s_, 1, x, y)
        pr.pr_hist_restrict(x, None, n, 1, g, ref[s_ + 1], ws)
        xs.append(x.clone())
    h = pr.pr_parareal_hist_create_chem(chem, sched, g, 2, 0, n, pr.PR_J_ADD, pr.PR_M_RESAMPLE, flags=pr.PR_PROFILE)
    try:
        err = np.zeros(2)
        pr.pr_parareal_hist_iterate(h, 1, rho_ref=ref, err_out=err)
        xr = torch.empty(n, dtype=torch.float64, device="cuda")
        rho = torch.empty(I, dtype=torch.float64, device="cuda")
        pr.pr_parareal_hist_state(h, 1, x=xr, rho=rho)
        assert torch.equal(xr, xs[1])
        assert torch.equal(rho, ref[1])
        for t in range(K + 1):
            pr.pr_parareal_hist_state(h, t, rho=rho)
            r = rho.cpu().numpy()
            assert np.all(r >= 0.0) and abs(r.sum() - 1.0) < 1e-12, t
        assert np.isfinite(err).all() and err[1] > 0.0
        ph, iters = pr.pr_parareal_hist_profile(h)
        assert iters == 1 and ph["fine"] > 0.0
    finally:
        pr.pr_parareal_hist_destroy(h)
