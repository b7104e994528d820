"""The restriction entry point that allocates nothing
(pr_restrict_quantiles_static, its workspace a static device array in the
library) against pr_restrict_quantiles with a caller workspace: every output
bit for bit, on two calls in a row, the second smaller than the first (the
array keeps the first call's contents), FP64 and FP32, and requests larger
than the array refused before any launch."""
import ctypes
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from tests import inputs

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


def _outputs(torch, k, n, nq, cells):
    z = lambda *shape, dt=torch.float64: torch.zeros(shape, dtype=dt, device="cuda")
    return dict(q=z(k, nq + 1), rank=z(k, n, dt=torch.int32), perm=z(k, n, dt=torch.int32), x_sorted=z(k, n),
                moments=z(k, 4), hist=z(k, cells, dt=torch.int32))


def _run_both(torch, x, prec, n, k, nq, grid):
    a = _outputs(torch, k, n, nq, grid.n_cells)
    b = _outputs(torch, k, n, nq, grid.n_cells)
    ws = torch.empty(pr.pr_restrict_workspace_size(n, k, prec), dtype=torch.uint8, device="cuda")
    pr.pr_restrict_quantiles(x, prec, n, k, nq, a["q"], ws, rank=a["rank"], perm=a["perm"], x_sorted=a["x_sorted"],
                             moments=a["moments"], hist=a["hist"], hist_grid=grid)
    pr.pr_restrict_quantiles_static(x, prec, n, k, nq, b["q"], rank=b["rank"], perm=b["perm"],
                                    x_sorted=b["x_sorted"], moments=b["moments"], hist=b["hist"], hist_grid=grid)
    torch.cuda.synchronize()
    for name in a:
        assert torch.equal(a[name], b[name]), name
    return b


@pytest.mark.parametrize("prec", [pr.PR_F64, pr.PR_F32])
def test_static_restriction_matches_the_workspace_form(torch_dev, prec):
    torch = torch_dev
    dt = torch.float64 if prec == pr.PR_F64 else torch.float32
    grid = pr.Grid(n_cells=64, n_q=100)
    # the largest request the array holds, then a smaller one with ties
    for k, n, seed in ((2, 1_048_576, 5), (3, 70_001, 6)):
        _say(f"static restriction prec={prec} k={k} n={n}")
        assert pr.pr_restrict_workspace_size(n, k, prec) <= pr.PR_STATIC_SCRATCH_BYTES
        x = torch.from_numpy(inputs.slow_values(seed, k, n)).to(dt).cuda()
        _run_both(torch, x, prec, n, k, 100, grid)


def test_static_restriction_refuses_requests_beyond_the_array(torch_dev):
    torch = torch_dev
    n, k = 1_048_576, 3
    assert pr.pr_restrict_workspace_size(n, k, pr.PR_F64) > pr.PR_STATIC_SCRATCH_BYTES
    L = pr.lib()
    buf = ctypes.c_void_p(16)
    rc = L.pr_restrict_quantiles_static(buf, pr.PR_F64, n, k, 100, None, buf, None, None, None, None, None, None)
    assert rc == -3
    assert "static scratch" in pr.pr_last_error()
