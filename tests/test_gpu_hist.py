"""GPU parity of the histogram-state path (iterators of Sec. 4, matchings of
Sec. 5, driver of Sec. 3.2) through the C ABI against the oracle on the same
seeded inputs: bitwise for the histograms, the iterators and the matchings
(the same formulas in the same order, exact fixed-point sums).  The driver
agrees within a tolerance: its coarse matrix-vector products sum in another
order than the oracle's, a 1e-16 difference that the union-of-levels
quantile iterator carries to ~1e-10 in the masses of tail cells (the oracle
alone moves by 6e-11 when its coarse sums run in reverse order), and that
the inverse cdf of the fast-marginal matching stretches by h / (cell mass)."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import coarse as OC
from oracle import histogram as H
from oracle import particles as OP

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


def _dev(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda() if dtype is None else \
        torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _grids(I, lo=-3.0, hi=3.0):
    return pr.Grid(n_cells=I, x_lo=lo, x_hi=hi), OC.Grid(I, lo, hi)


def _ensembles(k, n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, spread, (k, n))
    if n >= 3:
        x[:, :3] = [-9.0, 9.0, -3.0]  # outside the grid on both sides, and the left end
    return x


@pytest.mark.parametrize("k,n,I,weighted", [(1, 10_007, 64, False), (5, 4_099, 200, True), (3, 70_001, 1024, True),
                                            (2, 1, 17, False)])
def test_restrict_bitwise(torch_dev, k, n, I, weighted):
    torch = torch_dev
    _say(f"hist restrict k={k} n={n} I={I} w={weighted}")
    g, og = _grids(I)
    x = _ensembles(k, n, 1)
    rng = np.random.default_rng(2)
    w = rng.random((k, n)) ** 2 * 1e-3 if weighted else None
    rho = torch.empty((k, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_workspace_size(k, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_restrict(_dev(torch, x), _dev(torch, w) if weighted else None, n, k, g, rho, ws)
    got = rho.cpu().numpy()
    for s in range(k):
        ref = H.hist_restrict(x[s], w[s] if weighted else H.equal_weights(n), og)
        assert np.array_equal(got[s], ref), s


def _hists(rng, k, I, gaps):
    r = rng.random((k, I)) + 0.02
    if gaps:
        r[:, :3] = 0.0
        r[:, I // 2:I // 2 + 4] = 0.0
        r[:, -2:] = 0.0
    return r / r.sum(axis=1, keepdims=True)


def test_jump_quantile_long_decreasing_runs(torch_dev):
    """Fine histograms with all their mass in three cells (flat fine quantile
    functions) against smooth coarse ones that disagree: the reconstructed
    quantile function then decreases over long stretches of levels, the case
    whose monotone repair merges hundreds of values into one pool."""
    torch = torch_dev
    I, k = 1024, 4
    _say(f"hist jump quantile long runs I={I}")
    g, og = _grids(I)
    c = og.mids

    def gauss(mu, sd):
        r = np.exp(-0.5 * ((c - mu) / sd) ** 2)
        return r / r.sum()

    rc = np.stack([gauss(0.0, 1.0), gauss(0.5, 0.7), gauss(-1.0, 1.2), gauss(0.2, 0.5)])
    rcs = np.stack([gauss(0.3, 0.8), gauss(-0.2, 1.1), gauss(-0.5, 0.6), gauss(0.0, 0.9)])
    rf = np.zeros((k, I))
    for s, cells in enumerate([(300, 512, 700), (100, 101, 900), (512, 513, 514), (10, 600, 1000)]):
        rf[s, list(cells)] = [0.3, 0.4, 0.3]
    out = torch.empty((k, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_jump_workspace_size(k, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_jump(pr.PR_J_QUANTILE, _dev(torch, rc), _dev(torch, rf), _dev(torch, rcs), k, g, out, ws)
    got = out.cpu().numpy()
    for s in range(k):
        ref = H.jump(pr.PR_J_QUANTILE, rc[s], rf[s], rcs[s], og)
        assert np.array_equal(got[s], ref), (s, np.abs(got[s] - ref).max())


@pytest.mark.parametrize("kind", [pr.PR_J_ADD, pr.PR_J_MULT, pr.PR_J_ROT, pr.PR_J_QUANTILE])
@pytest.mark.parametrize("I,gaps", [(50, False), (200, True), (1024, True)])
def test_jump_bitwise(torch_dev, kind, I, gaps):
    torch = torch_dev
    _say(f"hist jump kind={kind} I={I} gaps={gaps}")
    g, og = _grids(I)
    rng = np.random.default_rng(kind * 7 + I)
    k = 6
    rc, rf, rcs = _hists(rng, k, I, gaps), _hists(rng, k, I, gaps), _hists(rng, k, I, gaps)
    rc[0] = rcs[0]  # the iterator property case
    rcs[1, 5:9] = 0.0  # cells without coarse support
    out = torch.empty((k, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_jump_workspace_size(k, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_jump(kind, _dev(torch, rc), _dev(torch, rf), _dev(torch, rcs), k, g, out, ws)
    got = out.cpu().numpy()
    for s in range(k):
        ref = H.jump(kind, rc[s], rf[s], rcs[s], og)
        assert np.array_equal(got[s], ref), (s, np.abs(got[s] - ref).max())


@pytest.mark.parametrize("kind", [pr.PR_M_MARGINAL, pr.PR_M_REWEIGHT, pr.PR_M_RESAMPLE, pr.PR_M_RESAMPLE_DET])
@pytest.mark.parametrize("k,n,I,one_prior", [(3, 5_003, 64, False), (2, 20_000, 1024, True)])
def test_match_bitwise(torch_dev, kind, k, n, I, one_prior):
    torch = torch_dev
    _say(f"hist match kind={kind} k={k} n={n} I={I} one_prior={one_prior}")
    g, og = _grids(I)
    kp = 1 if one_prior else k
    x = _ensembles(kp, n, 3, 0.7)
    rng = np.random.default_rng(4)
    y = rng.normal(0.0, 1.0, (kp, 1, n))
    w = rng.random((kp, n)) + 0.5
    w = w / w.sum(axis=1, keepdims=True)
    rp = np.stack([H.hist_restrict(x[s], w[s], og) for s in range(kp)])
    rt = _hists(rng, k, I, True)
    rt[0] = rp[0]  # identity case
    ws = torch.empty(pr.pr_hist_match_workspace_size(n, k, I), dtype=torch.uint8, device="cuda")
    xo = torch.full((k, n), np.nan, dtype=torch.float64, device="cuda")
    yo = torch.full((k, 1, n), np.nan, dtype=torch.float64, device="cuda")
    wo = torch.full((k, n), np.nan, dtype=torch.float64, device="cuda")
    rp_full = np.stack([rp[0 if one_prior else s] for s in range(k)])
    pr.pr_hist_match(kind, _dev(torch, rt), _dev(torch, rp_full), n, k, 1, g, _dev(torch, x), _dev(torch, y),
                     _dev(torch, w), 0 if one_prior else n, xo, yo, wo, ws, seed=11, instance=2, t_first=5)
    xg, yg, wg = xo.cpu().numpy(), yo.cpu().numpy(), wo.cpu().numpy()
    for s in range(k):
        p = 0 if one_prior else s
        xr, yr, wr = H.match(kind, rt[s], rp[p], (x[p], y[p], w[p]), og, 11, 2, 5 + s)
        if kind == pr.PR_M_MARGINAL:
            assert np.array_equal(xg[s], xr)
        elif kind == pr.PR_M_REWEIGHT:
            assert np.array_equal(wg[s], wr)
        else:
            assert np.array_equal(xg[s], xr) and np.array_equal(yg[s], yr) and np.array_equal(wg[s], wr)


@pytest.mark.parametrize("it", [pr.PR_J_ADD, pr.PR_J_MULT, pr.PR_J_ROT, pr.PR_J_QUANTILE])
@pytest.mark.parametrize("mt", [pr.PR_M_MARGINAL, pr.PR_M_REWEIGHT, pr.PR_M_RESAMPLE, pr.PR_M_RESAMPLE_DET])
def test_driver_matches_oracle(torch_dev, it, mt):
    torch = torch_dev
    _say(f"hist driver it={it} mt={mt}")
    n, K, T, dt, I = 3000, 4, 0.4, 1e-2, 40
    g, og = _grids(I, -2.5, 2.5)
    S = int(round(T / dt))
    sde = pr.Sde(lam=1.0, eps=0.1, beta=2.0)
    h = pr.pr_parareal_hist_create(sde, pr.Schedule(S, K, T / S), g, 5, 0, n, it, mt)
    osde = OP.Sde(lam=1.0, eps=0.1, beta=2.0)
    orc, hp = H.micmac_parareal_hist(osde, 5, 0, n, T, dt, K, og, it, mt)
    try:
        for k in range(3):
            if k > 0:
                pr.pr_parareal_hist_iterate(h, 1)
                orc.iterate()
            for t in range(K + 1):
                x = torch.empty(n, dtype=torch.float64, device="cuda")
                w = torch.empty(n, dtype=torch.float64, device="cuda")
                rho = torch.empty(I, dtype=torch.float64, device="cuda")
                pr.pr_parareal_hist_state(h, t, x=x, w=w, rho=rho)
                u = orc.u[t]
                x_tol, rho_tol = (1e-6, 1e-9) if it == pr.PR_J_QUANTILE else (1e-10, 1e-12)
                assert np.abs(x.cpu().numpy() - u.x).max() < x_tol, (k, t)
                assert np.abs(w.cpu().numpy() - u.w).max() < 1e-14, (k, t)
                assert np.abs(rho.cpu().numpy() - orc.rho[t]).max() < rho_tol, (k, t)
        assert pr.pr_parareal_hist_iteration(h) == 2
    finally:
        pr.pr_parareal_hist_destroy(h)


@pytest.mark.parametrize("it,mt", [(pr.PR_J_ADD, pr.PR_M_RESAMPLE), (pr.PR_J_QUANTILE, pr.PR_M_MARGINAL),
                                   (pr.PR_J_ROT, pr.PR_M_REWEIGHT)])
def test_driver_error_and_exactness(torch_dev, it, mt):
    """The L2 error of the new states' histograms against the serial fine
    run (computed by the library from a reference it is given) vanishes
    after N iterations (Sec. 3.3.3).  The states themselves are exact where
    the iterator's fixed point is exact (additive) or the matching leaves
    the slow variable alone (reweighting); the union-of-levels quantile
    iterator smears mass into empty interior cells of the fine histogram,
    which the fast-marginal matching turns into moves of particles inside
    their cells, so only its histograms are compared."""
    torch = torch_dev
    _say(f"hist driver error it={it} mt={mt}")
    n, K, T, dt, I = 4000, 4, 0.4, 1e-2, 20
    g, og = _grids(I, -2.0, 2.0)
    S = int(round(T / dt))
    sde = pr.Sde(lam=1.0, eps=0.1, beta=2.0)
    sched = pr.Schedule(S, K, T / S)
    # serial reference through the library's own kernels
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, 5, 0, n, x, y)
    ref = torch.empty((K + 1, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_workspace_size(1, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_restrict(x, None, n, 1, g, ref[0], ws)
    for s_ in range(K):
        pr.pr_fine_propagate(sde, sched, 5, 0, n, s_, 1, x, y)
        pr.pr_hist_restrict(x, None, n, 1, g, ref[s_ + 1], ws)
    h = pr.pr_parareal_hist_create(sde, sched, g, 5, 0, n, it, mt, flags=pr.PR_PROFILE)
    try:
        err = np.zeros(2 * K)
        pr.pr_parareal_hist_iterate(h, K, rho_ref=ref, err_out=err)
        assert err[-1] < 1e-12 and err[-2] < 1e-12, err
        ph, iters = pr.pr_parareal_hist_profile(h)
        assert iters == K and all(v >= 0 for v in ph.values())
        xr = torch.empty(n, dtype=torch.float64, device="cuda")
        pr.pr_parareal_hist_state(h, K, x=xr)
        if it != pr.PR_J_QUANTILE:
            assert torch.abs(xr - x).max().item() < 1e-12
    finally:
        pr.pr_parareal_hist_destroy(h)
