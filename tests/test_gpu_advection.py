"""GPU parity of the linear-advection study (Sec. 6, the linear advection
case) through the C ABI against the oracle: the exponentials of the
advection-diffusion coarse model, and the deterministic parareal on cell
masses for every iterator and biased coarse model (the oracle's coarse
products sum in another order than the library's, so masses agree within
1e-10, plus 100 times what the oracle itself moves when its products run in
reverse order; the iterators alone are compared bit for bit elsewhere)."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import advection as AD
from oracle import coarse as OC
from oracle import histogram as H

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


@pytest.mark.parametrize("eps,beta,I,K", [(1.0, 1.0, 800, 10), (2.0, 0.5, 300, 7), (0.5, 2.0, 1024, 64)])
def test_advection_exponential(torch_dev, eps, beta, I, K):
    torch = torch_dev
    _say(f"advection E eps={eps} beta={beta} I={I} K={K}")
    T = 1.0
    h = pr.pr_advection_coarse_create(eps, beta, pr.Schedule(100 * K, K, T / (100 * K)),
                                      pr.Grid(n_cells=I, x_lo=-8.0, x_hi=8.0))
    try:
        torch.cuda.synchronize()
        Eg = _copy_device(pr.pr_coarse_matrix(h, 0), I * I).reshape(I, I)
        Eo = AD.Propagator(OC.Grid(I, -8.0, 8.0), AD.Advection(eps, beta)).expm(T / K)
        assert np.abs(Eg - Eo).max() < 1e-12
        assert np.abs(Eg.sum(0) - 1).max() < 1e-12
    finally:
        pr.pr_coarse_destroy(h)


@pytest.mark.parametrize("it", [pr.PR_J_ADD, pr.PR_J_MULT, pr.PR_J_ROT, pr.PR_J_QUANTILE])
@pytest.mark.parametrize("eps_c,beta_c", [(1.0, 2.0), (2.0, 1.0), (1.0, 0.5)])
def test_fp_parareal_matches_oracle(torch_dev, it, eps_c, beta_c):
    torch = torch_dev
    _say(f"fp parareal it={it} coarse=({eps_c}, {beta_c})")
    I, K, T = 800, 10, 1.0
    grid, og = pr.Grid(n_cells=I, x_lo=-8.0, x_hi=8.0), OC.Grid(I, -8.0, 8.0)
    sched = pr.Schedule(100 * K, K, T / (100 * K))
    rho0 = AD.gaussian_cells(og, 2.0, 0.5)
    orc, serial, EF, EC = AD.fp_parareal(AD.Advection(), AD.Advection(eps_c, beta_c), og, rho0, T, K, it)
    alt, _, _, _ = AD.fp_parareal(AD.Advection(), AD.Advection(eps_c, beta_c), og, rho0, T, K, it)
    alt.fine = lambda n, u: np.maximum(EF[:, ::-1] @ u[::-1], 0.0)
    alt.coarse = lambda n, u: np.maximum(EC[:, ::-1] @ u[::-1], 0.0)
    hf = pr.pr_advection_coarse_create(1.0, 1.0, sched, grid)
    hc = pr.pr_advection_coarse_create(eps_c, beta_c, sched, grid)
    ref = torch.from_numpy(np.stack(serial)).cuda()
    # rounding differences of the coarse sums grow along the chain and over
    # the iterations (to ~2e-12 after three); a wrong operator, slice or
    # argument order moves the masses by 1e-3 or more
    base = 1e-10
    h = None
    try:
        h = pr.pr_parareal_fp_create(hf, hc, grid, torch.from_numpy(rho0).cuda(), it)
        rho = torch.empty(I, dtype=torch.float64, device="cuda")
        for k in range(4):
            if k > 0:
                err = np.zeros(2)
                pr.pr_parareal_fp_iterate(h, 1, rho_ref=ref, err_out=err)
                orc.iterate()
                alt.iterate()
                e_or = max(H.hist_error(orc.rho[n], serial[n]) for n in range(K + 1))
                assert abs(err[1] - e_or) < 1e-10 + 1e-6 * e_or, (k, err, e_or)
            for t in range(K + 1):
                pr.pr_parareal_fp_state(h, t, rho)
                tol = base + 100.0 * np.abs(alt.rho[t] - orc.rho[t]).max()
                assert np.abs(rho.cpu().numpy() - orc.rho[t]).max() < tol, (k, t)
        assert pr.pr_parareal_fp_iteration(h) == 3
        # exactness: after K iterations every state is the serial fine run, to
        # rounding (within 10 times the oracle's own distance to it: the
        # rotation iterator keeps its fixed point only to ~1e-10)
        pr.pr_parareal_fp_iterate(h, K - 3)
        for _ in range(K - 3):
            orc.iterate()
        for t in range(K + 1):
            pr.pr_parareal_fp_state(h, t, rho)
            tol = base + 10.0 * np.abs(orc.rho[t] - serial[t]).max()
            assert np.abs(rho.cpu().numpy() - serial[t]).max() < tol, t
    finally:
        if h is not None:
            pr.pr_parareal_fp_destroy(h)
        pr.pr_coarse_destroy(hf)
        pr.pr_coarse_destroy(hc)
