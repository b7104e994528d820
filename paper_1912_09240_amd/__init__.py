"""Python binding of the MI355X micro-macro parareal library (``libpr.so``).

Argument marshalling only: every function forwards to the C entry point of the
same name in ``include/pr.h``; all computation happens in the HIP kernels of
the library.  Tensors are passed by device pointer, streams as the raw
hipStream_t of ``torch.cuda`` (the current stream when none is given).
Importing this module does not need a GPU; calling into the library does, and
a missing library is an error, never a fallback.
"""
import ctypes
import os

__all__ = [
    "Sde", "Schedule", "Grid", "PrError", "lib", "available",
    "pr_version", "pr_last_error", "pr_draw_coupling", "pr_init_ensemble", "pr_fine_propagate",
    "pr_restrict_workspace_size", "pr_restrict_quantiles", "pr_restrict_quantiles_static", "PR_STATIC_SCRATCH_BYTES",
    "pr_match_quantiles", "pr_match_knots",
    "pr_coarse_create", "pr_coarse_fp_step", "pr_coarse_matrix", "pr_coarse_destroy", "pr_quantile_jump",
    "pr_parareal_create", "pr_parareal_iterate", "pr_parareal_state", "pr_parareal_iteration",
    "pr_parareal_knot_sorts", "pr_parareal_destroy", "pr_parareal_profile", "PR_F64", "PR_F32", "PR_REUSE_COARSE",
    "PR_SKIP_CONVERGED", "PR_PROFILE", "PHASES", "pr_fine_checkpoint", "pr_observables_workspace_size", "pr_observables",
    "pr_adjoint_workspace_size", "pr_fine_adjoint", "pr_draw_instances", "pr_parareal_batch_create",
    "pr_parareal_batch_iterate", "pr_parareal_batch_state", "pr_parareal_batch_info", "pr_parareal_batch_knot_sorts",
    "pr_parareal_batch_destroy",
    "PR_AUTOTUNE", "PR_LAUNCH_BATCHED", "PR_LAUNCH_GRAPH", "PR_LAUNCH_PER_INSTANCE",
    "PR_J_ADD", "PR_J_MULT", "PR_J_ROT", "PR_J_QUANTILE", "PR_M_MARGINAL", "PR_M_REWEIGHT", "PR_M_RESAMPLE",
    "PR_M_RESAMPLE_DET", "pr_hist_workspace_size", "pr_hist_restrict", "pr_hist_jump_workspace_size", "pr_hist_jump",
    "pr_hist_match_workspace_size", "pr_hist_match", "pr_parareal_hist_create", "pr_parareal_hist_iterate",
    "pr_parareal_hist_state", "pr_parareal_hist_iteration", "pr_parareal_hist_profile", "pr_parareal_hist_destroy",
    "Chem", "CHEM_K_DEFAULT", "pr_chem_init_ensemble", "pr_chem_fine_propagate", "pr_chem_mean_fast",
    "pr_chem_coarse_create", "pr_parareal_hist_create_chem", "pr_advection_coarse_create", "pr_parareal_fp_create",
    "pr_parareal_fp_iterate", "pr_parareal_fp_state", "pr_parareal_fp_iteration", "pr_parareal_fp_destroy",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpr.so")

PR_F64, PR_F32 = 64, 32
PR_STATIC_SCRATCH_BYTES = 64 << 20
PR_REUSE_COARSE, PR_SKIP_CONVERGED, PR_PROFILE, PR_AUTOTUNE = 1, 2, 4, 8
PR_LAUNCH_BATCHED, PR_LAUNCH_GRAPH, PR_LAUNCH_PER_INSTANCE = 0, 1, 2
PR_J_ADD, PR_J_MULT, PR_J_ROT, PR_J_QUANTILE = 0, 1, 2, 3
PR_M_MARGINAL, PR_M_REWEIGHT, PR_M_RESAMPLE, PR_M_RESAMPLE_DET = 0, 1, 2, 3
PHASES = ("fine", "restrict_fine", "coarse", "chain", "match", "restrict_new")

_c_int, _c_i64, _c_u32, _c_u64, _c_dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_vp = ctypes.c_void_p


class _CSde(ctypes.Structure):
    _fields_ = [("d_fast", _c_int), ("precision", _c_int), ("lambda_", _c_dbl), ("eps", _c_dbl),
                ("beta", _c_dbl), ("c3", _c_dbl), ("c1", _c_dbl), ("a", _vp)]


class _CSchedule(ctypes.Structure):
    _fields_ = [("total_steps", _c_i64), ("n_slices", _c_int), ("dt", _c_dbl)]


class _CGrid(ctypes.Structure):
    _fields_ = [("n_cells", _c_int), ("x_lo", _c_dbl), ("x_hi", _c_dbl), ("n_q", _c_int)]


class Sde:
    """Slow-fast SDE parameters (pr_sde).  ``a`` is a device tensor of d
    doubles or None (all ones)."""

    def __init__(self, lam=1.0, eps=0.1, beta=2.0, c3=1.0, c1=-1.0, d=1, precision=PR_F64, a=None):
        self.lam, self.eps, self.beta, self.c3, self.c1 = lam, eps, beta, c3, c1
        self.d, self.precision, self.a = d, precision, a

    def c(self):
        return _CSde(self.d, self.precision, self.lam, self.eps, self.beta, self.c3, self.c1,
                     _ptr(self.a) if self.a is not None else None)


class Schedule:
    """pr_schedule: S fine steps of dt in n_slices slices."""

    def __init__(self, total_steps, n_slices, dt):
        self.total_steps, self.n_slices, self.dt = int(total_steps), int(n_slices), float(dt)

    def c(self):
        return _CSchedule(self.total_steps, self.n_slices, self.dt)


class Grid:
    """pr_grid: n_cells on [x_lo, x_hi], knots at j/n_q."""

    def __init__(self, n_cells=200, x_lo=-3.0, x_hi=3.0, n_q=100):
        self.n_cells, self.x_lo, self.x_hi, self.n_q = int(n_cells), float(x_lo), float(x_hi), int(n_q)

    def c(self):
        return _CGrid(self.n_cells, self.x_lo, self.x_hi, self.n_q)


class _CChem(ctypes.Structure):
    _fields_ = [("tau_x", _c_dbl), ("eps", _c_dbl), ("k", _c_dbl * 6), ("x0_mean", _c_dbl), ("x0_sd", _c_dbl),
                ("y0_mean", _c_dbl), ("y0_sd", _c_dbl)]


CHEM_K_DEFAULT = (60.0, 1.0, 4.8e-3, 0.666e-5, 0.833, 1.0)


class Chem:
    """Chemical-reaction system parameters (pr_chem): Table 1 defaults with
    k3 = 0.666e-5 (bistable fast variable)."""

    def __init__(self, tau_x=25.0, eps=2.5e-2, k=CHEM_K_DEFAULT, x0=(100.0, 20.0), y0=(100.0, 20.0)):
        self.tau_x, self.eps = float(tau_x), float(eps)
        self.k = tuple(float(v) for v in k)
        self.x0, self.y0 = tuple(x0), tuple(y0)

    def c(self):
        s = _CChem()
        s.tau_x, s.eps = self.tau_x, self.eps
        for i in range(6):
            s.k[i] = self.k[i]
        s.x0_mean, s.x0_sd = self.x0
        s.y0_mean, s.y0_sd = self.y0
        return s


class PrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pr status {status}: {msg}")
        self.status = status


_LIB = None

_SIGS = {
    "pr_last_error": (ctypes.c_char_p, []),
    "pr_version": (_c_int, []),
    "pr_draw_coupling": (_c_int, [_c_u64, _c_u32, _c_int, _vp, _vp]),
    "pr_init_ensemble": (_c_int, [ctypes.POINTER(_CSde), _c_u64, _c_u32, _c_i64, _vp, _vp, _vp]),
    "pr_fine_propagate": (_c_int, [ctypes.POINTER(_CSde), ctypes.POINTER(_CSchedule), _c_u64, _c_u32, _c_i64,
                                   _c_int, _c_int, _vp, _vp, _vp]),
    "pr_restrict_workspace_size": (ctypes.c_size_t, [_c_i64, _c_int, _c_int]),
    "pr_restrict_quantiles": (_c_int, [_vp, _c_int, _c_i64, _c_int, _c_int, ctypes.POINTER(_CGrid), _vp, _vp, _vp,
                                       _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "pr_restrict_quantiles_static": (_c_int, [_vp, _c_int, _c_i64, _c_int, _c_int, ctypes.POINTER(_CGrid), _vp, _vp,
                                              _vp, _vp, _vp, _vp, _vp]),
    "pr_match_quantiles": (_c_int, [_vp, _vp, _vp, _c_i64, _c_int, _c_int, _vp, _vp, _c_int, _vp]),
    "pr_match_knots": (_c_int, [_vp, _vp, _c_i64, _c_int, _c_int, _c_int, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    "pr_coarse_create": (_c_int, [ctypes.POINTER(_CSde), ctypes.POINTER(_CSchedule), ctypes.POINTER(_CGrid), _vp,
                                  ctypes.POINTER(_vp)]),
    "pr_coarse_fp_step": (_c_int, [_vp, _c_int, _c_int, _vp, _vp, _vp, _vp]),
    "pr_coarse_matrix": (_c_int, [_vp, _c_int, ctypes.POINTER(_vp)]),
    "pr_coarse_destroy": (_c_int, [_vp]),
    "pr_quantile_jump": (_c_int, [_vp, _vp, _vp, _c_int, _c_int, _vp, _vp]),
    "pr_parareal_create": (_c_int, [ctypes.POINTER(_CSde), ctypes.POINTER(_CSchedule), ctypes.POINTER(_CGrid),
                                    _c_u64, _c_u32, _c_i64, _c_int, _vp, ctypes.POINTER(_vp)]),
    "pr_parareal_iterate": (_c_int, [_vp, _c_int, _vp, _vp, _vp]),
    "pr_parareal_state": (_c_int, [_vp, _c_int, _vp, _vp, _vp, _vp]),
    "pr_parareal_iteration": (_c_int, [_vp]),
    "pr_parareal_knot_sorts": (_c_int, [_vp]),
    "pr_parareal_destroy": (_c_int, [_vp]),
    "pr_parareal_profile": (_c_int, [_vp, ctypes.POINTER(_c_dbl), ctypes.POINTER(_c_int)]),
    "pr_fine_checkpoint": (_c_int, [ctypes.POINTER(_CSde), ctypes.POINTER(_CSchedule), _c_u64, _c_u32, _c_i64,
                                    _vp, _vp, _vp, _c_int, _vp]),
    "pr_observables_workspace_size": (ctypes.c_size_t, [_c_i64]),
    "pr_observables": (_c_int, [_vp, _c_i64, ctypes.POINTER(_c_dbl), _c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "pr_adjoint_workspace_size": (ctypes.c_size_t, [_c_i64, _c_int, _c_int]),
    "pr_draw_instances": (_c_int, [_c_u64, _c_int, _vp, _vp]),
    "pr_parareal_batch_create": (_c_int, [_c_int, _vp, _vp, _vp, ctypes.POINTER(_CGrid), _c_u64, _vp, _c_int, _vp,
                                          ctypes.POINTER(_vp)]),
    "pr_parareal_batch_iterate": (_c_int, [_vp, _c_int, _c_int, ctypes.POINTER(_c_dbl), _vp]),
    "pr_parareal_batch_state": (_c_int, [_vp, _c_int, _c_int, _vp, _vp, _vp, _vp]),
    "pr_parareal_batch_info": (_c_int, [_vp, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_i64),
                                        ctypes.POINTER(_c_i64), ctypes.POINTER(_c_int)]),
    "pr_parareal_batch_knot_sorts": (_c_int, [_vp, ctypes.POINTER(_c_i64)]),
    "pr_parareal_batch_destroy": (_c_int, [_vp]),
    "pr_fine_adjoint": (_c_int, [ctypes.POINTER(_CSde), ctypes.POINTER(_CSchedule), _c_u64, _c_u32, _c_i64, _vp,
                                 _c_int, _vp, _vp, _c_int, _c_int, _vp, _vp, ctypes.c_size_t, _vp]),
    "pr_hist_workspace_size": (ctypes.c_size_t, [_c_int, _c_int]),
    "pr_hist_restrict": (_c_int, [_vp, _vp, _c_i64, _c_int, ctypes.POINTER(_CGrid), _vp, _vp, ctypes.c_size_t, _vp]),
    "pr_hist_jump_workspace_size": (ctypes.c_size_t, [_c_int, _c_int]),
    "pr_hist_jump": (_c_int, [_c_int, _vp, _vp, _vp, _c_int, ctypes.POINTER(_CGrid), _vp, _vp, ctypes.c_size_t, _vp]),
    "pr_hist_match_workspace_size": (ctypes.c_size_t, [_c_i64, _c_int, _c_int]),
    "pr_hist_match": (_c_int, [_c_int, _vp, _vp, _c_i64, _c_int, _c_int, ctypes.POINTER(_CGrid), _vp, _vp, _vp, _c_i64,
                               _vp, _vp, _vp, _c_u64, _c_u32, _c_int, _vp, ctypes.c_size_t, _vp]),
    "pr_parareal_hist_create": (_c_int, [ctypes.POINTER(_CSde), ctypes.POINTER(_CSchedule), ctypes.POINTER(_CGrid),
                                         _c_u64, _c_u32, _c_i64, _c_int, _c_int, _c_int, _vp, ctypes.POINTER(_vp)]),
    "pr_parareal_hist_iterate": (_c_int, [_vp, _c_int, _vp, _vp, _vp]),
    "pr_parareal_hist_state": (_c_int, [_vp, _c_int, _vp, _vp, _vp, _vp, _vp]),
    "pr_parareal_hist_iteration": (_c_int, [_vp]),
    "pr_parareal_hist_profile": (_c_int, [_vp, ctypes.POINTER(_c_dbl), ctypes.POINTER(_c_int)]),
    "pr_parareal_hist_destroy": (_c_int, [_vp]),
    "pr_chem_init_ensemble": (_c_int, [ctypes.POINTER(_CChem), _c_u64, _c_u32, _c_i64, _vp, _vp, _vp]),
    "pr_chem_fine_propagate": (_c_int, [ctypes.POINTER(_CChem), ctypes.POINTER(_CSchedule), _c_u64, _c_u32, _c_i64,
                                        _c_int, _c_int, _vp, _vp, _vp]),
    "pr_chem_mean_fast": (_c_int, [ctypes.POINTER(_CChem), ctypes.POINTER(_c_dbl)]),
    "pr_chem_coarse_create": (_c_int, [ctypes.POINTER(_CChem), ctypes.POINTER(_CSchedule), ctypes.POINTER(_CGrid),
                                       _vp, ctypes.POINTER(_vp)]),
    "pr_parareal_hist_create_chem": (_c_int, [ctypes.POINTER(_CChem), ctypes.POINTER(_CSchedule),
                                              ctypes.POINTER(_CGrid), _c_u64, _c_u32, _c_i64, _c_int, _c_int, _c_int,
                                              _vp, ctypes.POINTER(_vp)]),
    "pr_advection_coarse_create": (_c_int, [_c_dbl, _c_dbl, ctypes.POINTER(_CSchedule), ctypes.POINTER(_CGrid), _vp,
                                            ctypes.POINTER(_vp)]),
    "pr_parareal_fp_create": (_c_int, [_vp, _vp, ctypes.POINTER(_CGrid), _vp, _c_int, _c_int, _vp,
                                       ctypes.POINTER(_vp)]),
    "pr_parareal_fp_iterate": (_c_int, [_vp, _c_int, _vp, _vp, _vp]),
    "pr_parareal_fp_state": (_c_int, [_vp, _c_int, _vp, _vp]),
    "pr_parareal_fp_iteration": (_c_int, [_vp]),
    "pr_parareal_fp_destroy": (_c_int, [_vp]),
}


def available():
    return os.path.exists(LIB_PATH)


def lib():
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run paper_1912_09240_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status):
    if status != 0:
        raise PrError(status, lib().pr_last_error().decode())


def pr_version():
    return lib().pr_version()


def pr_last_error():
    return lib().pr_last_error().decode()


def pr_draw_coupling(seed, instance, d, a, stream=None):
    _check(lib().pr_draw_coupling(seed, instance, d, _ptr(a), _stream(stream)))


def pr_init_ensemble(sde, seed, instance, n, x, y, stream=None):
    s = sde.c()
    _check(lib().pr_init_ensemble(ctypes.byref(s), seed, instance, n, _ptr(x), _ptr(y), _stream(stream)))


def pr_fine_propagate(sde, sched, seed, instance, n, slice_first, slice_count, x, y, stream=None):
    s, c = sde.c(), sched.c()
    _check(lib().pr_fine_propagate(ctypes.byref(s), ctypes.byref(c), seed, instance, n, slice_first, slice_count,
                                   _ptr(x), _ptr(y), _stream(stream)))


def pr_restrict_workspace_size(n, k, precision=PR_F64):
    return lib().pr_restrict_workspace_size(n, k, precision)


def pr_restrict_quantiles(x, precision, n, k, n_q, q, ws, rank=None, perm=None, x_sorted=None, moments=None,
                          hist=None, hist_grid=None, stream=None):
    g = ctypes.byref(hist_grid.c()) if hist_grid is not None else None
    nbytes = ws.numel() * ws.element_size()
    _check(lib().pr_restrict_quantiles(_ptr(x), precision, n, k, n_q, g, _ptr(q), _ptr(rank), _ptr(perm),
                                       _ptr(x_sorted), _ptr(moments), _ptr(hist), _ptr(ws), nbytes, _stream(stream)))


def pr_restrict_quantiles_static(x, precision, n, k, n_q, q, rank=None, perm=None, x_sorted=None, moments=None,
                                 hist=None, hist_grid=None, stream=None):
    g = ctypes.byref(hist_grid.c()) if hist_grid is not None else None
    _check(lib().pr_restrict_quantiles_static(_ptr(x), precision, n, k, n_q, g, _ptr(q), _ptr(rank), _ptr(perm),
                                              _ptr(x_sorted), _ptr(moments), _ptr(hist), _stream(stream)))


def pr_match_quantiles(q_target, q_prior, rank, n, k, n_q, x_prior, x_out, precision=PR_F64, stream=None):
    _check(lib().pr_match_quantiles(_ptr(q_target), _ptr(q_prior), _ptr(rank), n, k, n_q, _ptr(x_prior),
                                    _ptr(x_out), precision, _stream(stream)))


def pr_match_knots(q_target, q_prior, n, k, n_q, ws, q_out, flag, precision=PR_F64, stream=None):
    nbytes = ws.numel() * ws.element_size()
    _check(lib().pr_match_knots(_ptr(q_target), _ptr(q_prior), n, k, n_q, precision, _ptr(ws), nbytes, _ptr(q_out),
                                _ptr(flag), _stream(stream)))


def pr_coarse_create(sde, sched, grid, stream=None):
    h = _vp()
    s, c, g = sde.c(), sched.c(), grid.c()
    _check(lib().pr_coarse_create(ctypes.byref(s), ctypes.byref(c), ctypes.byref(g), _stream(stream),
                                  ctypes.byref(h)))
    return h


def pr_coarse_fp_step(h, slice_first, slice_count, q_in, q_out, rho_out=None, stream=None):
    _check(lib().pr_coarse_fp_step(h, slice_first, slice_count, _ptr(q_in), _ptr(q_out), _ptr(rho_out),
                                   _stream(stream)))


def pr_coarse_matrix(h, slice_index):
    p = _vp()
    _check(lib().pr_coarse_matrix(h, slice_index, ctypes.byref(p)))
    return p.value


def pr_coarse_destroy(h):
    _check(lib().pr_coarse_destroy(h))


def pr_quantile_jump(q_c_next, q_f, q_c_star, k, n_q, q_out, stream=None):
    _check(lib().pr_quantile_jump(_ptr(q_c_next), _ptr(q_f), _ptr(q_c_star), k, n_q, _ptr(q_out), _stream(stream)))


def pr_parareal_create(sde, sched, grid, seed, instance, n, flags=0, stream=None):
    h = _vp()
    s, c, g = sde.c(), sched.c(), grid.c()
    _check(lib().pr_parareal_create(ctypes.byref(s), ctypes.byref(c), ctypes.byref(g), seed, instance, n, flags,
                                    _stream(stream), ctypes.byref(h)))
    return h


def pr_parareal_iterate(h, n_iter, q_ref=None, err_out=None, stream=None):
    """err_out: a host buffer (e.g. a numpy float64 array of 2*n_iter) or None."""
    ep = None
    if err_out is not None:
        ep = err_out.ctypes.data_as(_vp) if hasattr(err_out, "ctypes") else _ptr(err_out)
    _check(lib().pr_parareal_iterate(h, n_iter, _ptr(q_ref), ep, _stream(stream)))


def pr_parareal_state(h, t, x=None, y=None, q=None, stream=None):
    _check(lib().pr_parareal_state(h, t, _ptr(x), _ptr(y), _ptr(q), _stream(stream)))


def pr_parareal_iteration(h):
    return lib().pr_parareal_iteration(h)


def pr_parareal_knot_sorts(h):
    return lib().pr_parareal_knot_sorts(h)


def pr_parareal_destroy(h):
    _check(lib().pr_parareal_destroy(h))


def pr_parareal_profile(h):
    """{phase name: summed device ms}, number of timed iterations."""
    arr = (_c_dbl * len(PHASES))()
    it = _c_int()
    _check(lib().pr_parareal_profile(h, arr, ctypes.byref(it)))
    return dict(zip(PHASES, list(arr))), it.value


def pr_fine_checkpoint(sde, sched, seed, instance, n, x, y, ckpt, ckpt_every, stream=None):
    s, c = sde.c(), sched.c()
    _check(lib().pr_fine_checkpoint(ctypes.byref(s), ctypes.byref(c), seed, instance, n, _ptr(x), _ptr(y),
                                    _ptr(ckpt), ckpt_every, _stream(stream)))


def pr_observables_workspace_size(n):
    return lib().pr_observables_workspace_size(n)


def pr_observables(x, n, alpha, obs, ws, seed_x=None, stream=None):
    a = (_c_dbl * max(1, len(alpha)))(*alpha)
    nbytes = ws.numel() * ws.element_size()
    _check(lib().pr_observables(_ptr(x), n, a, len(alpha), _ptr(obs), _ptr(seed_x), _ptr(ws), nbytes,
                                _stream(stream)))


def pr_adjoint_workspace_size(n, ckpt_every, n_seed):
    return lib().pr_adjoint_workspace_size(n, ckpt_every, n_seed)


def pr_fine_adjoint(sde, sched, seed, instance, n, ckpt, ckpt_every, seed_x, n_seed, grad, ws, seed_y=None,
                    from_initial=True, stream=None):
    s, c = sde.c(), sched.c()
    nbytes = ws.numel() * ws.element_size()
    _check(lib().pr_fine_adjoint(ctypes.byref(s), ctypes.byref(c), seed, instance, n, _ptr(ckpt), ckpt_every,
                                 _ptr(seed_x), _ptr(seed_y), n_seed, 1 if from_initial else 0, _ptr(grad), _ptr(ws),
                                 nbytes, _stream(stream)))


def pr_draw_instances(seed, count, out, stream=None):
    """out: device float64 tensor [count][4] <- (eps, lambda, log2 n, slices)."""
    _check(lib().pr_draw_instances(seed, count, _ptr(out), _stream(stream)))


def pr_parareal_batch_create(sdes, scheds, ns, grid, seed, instances=None, flags=0, stream=None):
    B = len(sdes)
    S = (_CSde * B)(*[s.c() for s in sdes])
    C = (_CSchedule * B)(*[c.c() for c in scheds])
    N = (_c_i64 * B)(*ns)
    ids = (_c_u32 * B)(*instances) if instances is not None else None
    g = grid.c()
    h = _vp()
    _check(lib().pr_parareal_batch_create(B, ctypes.cast(S, _vp), ctypes.cast(C, _vp), ctypes.cast(N, _vp),
                                          ctypes.byref(g), seed, ctypes.cast(ids, _vp) if ids is not None else None,
                                          flags, _stream(stream), ctypes.byref(h)))
    return h


def pr_parareal_batch_iterate(h, n_iter, mode=PR_LAUNCH_BATCHED, timed=False, stream=None):
    """Returns the device time of the iterations in ms when timed."""
    ms = _c_dbl(0.0)
    _check(lib().pr_parareal_batch_iterate(h, n_iter, mode, ctypes.byref(ms) if timed else None, _stream(stream)))
    return ms.value if timed else None


def pr_parareal_batch_state(h, inst, t, x=None, y=None, q=None, stream=None):
    _check(lib().pr_parareal_batch_state(h, inst, t, _ptr(x), _ptr(y), _ptr(q), _stream(stream)))


def pr_parareal_batch_info(h):
    b, p, u, w, sp = _c_int(), _c_int(), _c_i64(), _c_i64(), _c_int()
    _check(lib().pr_parareal_batch_info(h, ctypes.byref(b), ctypes.byref(p), ctypes.byref(u), ctypes.byref(w),
                                        ctypes.byref(sp)))
    return dict(block=b.value, ppt=p.value, units=u.value, particle_steps=w.value, split_sort=bool(sp.value))


def pr_parareal_batch_knot_sorts(h):
    """(batched iterations whose new knots needed a sort, ensembles sorted)."""
    segs = _c_i64(0)
    n = lib().pr_parareal_batch_knot_sorts(h, ctypes.byref(segs))
    return n, segs.value


def pr_parareal_batch_destroy(h):
    _check(lib().pr_parareal_batch_destroy(h))


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def pr_hist_workspace_size(k, n_cells):
    return lib().pr_hist_workspace_size(k, n_cells)


def pr_hist_restrict(x, w, n, k, grid, rho, ws, stream=None):
    g = grid.c()
    _check(lib().pr_hist_restrict(_ptr(x), _ptr(w), n, k, ctypes.byref(g), _ptr(rho), _ptr(ws), _nbytes(ws),
                                  _stream(stream)))


def pr_hist_jump_workspace_size(k, n_cells):
    return lib().pr_hist_jump_workspace_size(k, n_cells)


def pr_hist_jump(kind, rho_c, rho_f, rho_cs, k, grid, rho_out, ws=None, stream=None):
    g = grid.c()
    _check(lib().pr_hist_jump(kind, _ptr(rho_c), _ptr(rho_f), _ptr(rho_cs), k, ctypes.byref(g), _ptr(rho_out),
                              _ptr(ws), _nbytes(ws), _stream(stream)))


def pr_hist_match_workspace_size(n, k, n_cells):
    return lib().pr_hist_match_workspace_size(n, k, n_cells)


def pr_hist_match(kind, rho_t, rho_p, n, k, d, grid, x, y, w, prior_stride, x_out, y_out, w_out, ws, seed=0,
                  instance=0, t_first=0, stream=None):
    g = grid.c()
    _check(lib().pr_hist_match(kind, _ptr(rho_t), _ptr(rho_p), n, k, d, ctypes.byref(g), _ptr(x), _ptr(y), _ptr(w),
                               prior_stride, _ptr(x_out), _ptr(y_out), _ptr(w_out), seed, instance, t_first, _ptr(ws),
                               _nbytes(ws), _stream(stream)))


def pr_parareal_hist_create(sde, sched, grid, seed, instance, n, iterator, matching, flags=0, stream=None):
    s, c, g = sde.c(), sched.c(), grid.c()
    h = _vp()
    _check(lib().pr_parareal_hist_create(ctypes.byref(s), ctypes.byref(c), ctypes.byref(g), seed, instance, n,
                                         iterator, matching, flags, _stream(stream), ctypes.byref(h)))
    return h


def pr_parareal_hist_iterate(h, n_iter, rho_ref=None, err_out=None, stream=None):
    """err_out: host float64 numpy array of 2 * n_iter (error at N, max over n)."""
    _check(lib().pr_parareal_hist_iterate(h, n_iter, _ptr(rho_ref),
                                          err_out.ctypes.data_as(_vp) if err_out is not None else None,
                                          _stream(stream)))


def pr_parareal_hist_state(h, t, x=None, y=None, w=None, rho=None, stream=None):
    _check(lib().pr_parareal_hist_state(h, t, _ptr(x), _ptr(y), _ptr(w), _ptr(rho), _stream(stream)))


def pr_parareal_hist_iteration(h):
    return lib().pr_parareal_hist_iteration(h)


def pr_parareal_hist_profile(h):
    ms = (_c_dbl * len(PHASES))()
    it = _c_int(0)
    _check(lib().pr_parareal_hist_profile(h, ms, ctypes.byref(it)))
    return dict(zip(PHASES, list(ms))), it.value


def pr_parareal_hist_destroy(h):
    _check(lib().pr_parareal_hist_destroy(h))


def pr_chem_init_ensemble(chem, seed, instance, n, x, y, stream=None):
    c = chem.c()
    _check(lib().pr_chem_init_ensemble(ctypes.byref(c), seed, instance, n, _ptr(x), _ptr(y), _stream(stream)))


def pr_chem_fine_propagate(chem, sched, seed, instance, n, slice_first, slice_count, x, y, stream=None):
    c, s = chem.c(), sched.c()
    _check(lib().pr_chem_fine_propagate(ctypes.byref(c), ctypes.byref(s), seed, instance, n, slice_first, slice_count,
                                        _ptr(x), _ptr(y), _stream(stream)))


def pr_chem_mean_fast(chem):
    c = chem.c()
    v = _c_dbl(0.0)
    _check(lib().pr_chem_mean_fast(ctypes.byref(c), ctypes.byref(v)))
    return v.value


def pr_chem_coarse_create(chem, sched, grid, stream=None):
    c, s, g = chem.c(), sched.c(), grid.c()
    h = _vp()
    _check(lib().pr_chem_coarse_create(ctypes.byref(c), ctypes.byref(s), ctypes.byref(g), _stream(stream),
                                       ctypes.byref(h)))
    return h


def pr_parareal_hist_create_chem(chem, sched, grid, seed, instance, n, iterator, matching, flags=0, stream=None):
    c, s, g = chem.c(), sched.c(), grid.c()
    h = _vp()
    _check(lib().pr_parareal_hist_create_chem(ctypes.byref(c), ctypes.byref(s), ctypes.byref(g), seed, instance, n,
                                              iterator, matching, flags, _stream(stream), ctypes.byref(h)))
    return h


def pr_advection_coarse_create(eps, beta, sched, grid, stream=None):
    s, g = sched.c(), grid.c()
    h = _vp()
    _check(lib().pr_advection_coarse_create(eps, beta, ctypes.byref(s), ctypes.byref(g), _stream(stream),
                                            ctypes.byref(h)))
    return h


def pr_parareal_fp_create(fine, coarse, grid, rho0, iterator, flags=0, stream=None):
    g = grid.c()
    h = _vp()
    _check(lib().pr_parareal_fp_create(fine, coarse, ctypes.byref(g), _ptr(rho0), iterator, flags, _stream(stream),
                                       ctypes.byref(h)))
    return h


def pr_parareal_fp_iterate(h, n_iter, rho_ref=None, err_out=None, stream=None):
    """err_out: host float64 numpy array of 2 * n_iter (error at N, max over n)."""
    _check(lib().pr_parareal_fp_iterate(h, n_iter, _ptr(rho_ref),
                                        err_out.ctypes.data_as(_vp) if err_out is not None else None,
                                        _stream(stream)))


def pr_parareal_fp_state(h, t, rho, stream=None):
    _check(lib().pr_parareal_fp_state(h, t, _ptr(rho), _stream(stream)))


def pr_parareal_fp_iteration(h):
    return lib().pr_parareal_fp_iteration(h)


def pr_parareal_fp_destroy(h):
    _check(lib().pr_parareal_fp_destroy(h))
