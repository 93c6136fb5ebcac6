"""ctypes binding of libsgpdeconv.so (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor
placement and dtype, converts keyword parameters into ``sgp_params`` and
turns return codes into exceptions.  PyTorch provides device memory and the
current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsgpdeconv.so")

TRACE_COLS = 20
TRACE_FIELDS = ["k", "alpha", "gd", "backtracks", "lam", "J", "a", "c1", "c2", "e",
                "a1", "a2", "br1", "br2", "alt", "tau", "alpha_next", "flux_mu"]

STOP_FIXED, STOP_CONV, STOP_DISCREPANCY, STOP_RMSE = 1, 2, 4, 8
INIT_FLAT, INIT_ZERO, INIT_DATA, INIT_USER, INIT_WARM = 0, 1, 2, 3, 4
REASONS = {0: "maxiter", 1: "convergence", 2: "discrepancy", 3: "rmse", 4: "stationary", 5: "armijo",
           6: "numeric"}


class SgpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sgpdeconv error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int), ("stop", ctypes.c_int), ("tol", ctypes.c_double),
        ("disc_target", ctypes.c_double), ("init", ctypes.c_int), ("f0", ctypes.c_void_p),
        ("beta", ctypes.c_double), ("theta", ctypes.c_double), ("alpha0", ctypes.c_double),
        ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("tau1", ctypes.c_double),
        ("m_alpha", ctypes.c_int), ("n_bb2_only", ctypes.c_int), ("auto_bounds", ctypes.c_int),
        ("L1", ctypes.c_double), ("L2", ctypes.c_double), ("flux_constraint", ctypes.c_int),
        ("flux", ctypes.c_double), ("sigma_R", ctypes.c_double), ("max_backtracks", ctypes.c_int),
        ("trace", ctypes.c_void_p), ("rl_alpha", ctypes.c_double), ("f_true", ctypes.c_void_p),
        ("rl_line_search", ctypes.c_int), ("rl_lambda_cap", ctypes.c_double),
    ]


class _Report(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int), ("stop_reason", ctypes.c_int), ("backtracks", ctypes.c_int),
        ("used_fallback", ctypes.c_int), ("kl", ctypes.c_double), ("discrepancy", ctypes.c_double),
        ("flux", ctypes.c_double), ("L1", ctypes.c_double), ("L2", ctypes.c_double),
        ("seconds", ctypes.c_double), ("flux_unconverged", ctypes.c_int),
    ]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("g", ctypes.c_void_p), ("psf", ctypes.c_void_p), ("b_map", ctypes.c_void_p),
        ("b_const", ctypes.c_void_p), ("p", ctypes.c_int), ("ny", ctypes.c_int), ("nx", ctypes.c_int),
        ("NY", ctypes.c_int), ("NX", ctypes.c_int), ("oy", ctypes.c_int), ("ox", ctypes.c_int),
        ("boundary", ctypes.c_int),
    ]


KIND_RL, KIND_SGP, KIND_OSEM = 0, 1, 2
KCLASSES = ["row_dir", "col_conv", "row_ad", "armijo_more", "row_upd", "col_corr", "row_grad",
            "row_ratio", "row_rlupd", "row_fin"]

EXPORTS = [
    "sgp_params_init", "rl_deconv", "sgp_deconv", "sgp_deconv_noalloc", "sgp_multi_deconv", "rl_multi_deconv",
    "sgp_boundary_deconv", "rl_boundary_deconv", "sgp_apply_operator", "sgp_release_cache",
    "sgp_strerror", "sgp_last_error", "sgp_solver_create", "sgp_solver_step", "sgp_solver_prepare",
    "sgp_solver_report", "sgp_solver_gradient",
    "sgp_solver_set_timing", "sgp_solver_set_graph", "sgp_solver_timing", "sgp_solver_destroy",
    "sgp_steplength_rule", "sgp_batch_deconv", "osem_deconv", "osem_boundary_deconv", "sgp_mosaic_deconv",
    "sgp_cnn_num_params", "sgp_cnn_create", "sgp_cnn_get_params", "sgp_cnn_infer", "sgp_cnn_loss_grad",
    "sgp_cnn_adam_step", "sgp_cnn_train_step", "sgp_cnn_destroy",
    "sgp_tile_info", "sgp_set_tile_schedule", "sgp_get_tile_schedule", "sgp_save_tile_schedule",
    "sgp_load_tile_schedule", "sgp_autotune", "sgp_flux_multiplier",
]

_lib = None


def load():
    """Loads the library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1210_2258_amd.build.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, R, vp, i, f, d = (ctypes.POINTER(_Params), ctypes.POINTER(_Report), ctypes.c_void_p,
                         ctypes.c_int, ctypes.c_float, ctypes.c_double)
    lib.sgp_params_init.argtypes = [P]
    for name in ("rl_deconv", "sgp_deconv", "sgp_deconv_noalloc"):
        getattr(lib, name).argtypes = [vp, vp, vp, f, i, i, P, vp, R, vp]
    for name in ("sgp_multi_deconv", "rl_multi_deconv", "osem_deconv"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp, i, i, i, P, vp, R, vp]
    for name in ("sgp_boundary_deconv", "rl_boundary_deconv", "osem_boundary_deconv"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp, i, i, i, i, i, i, i, P, vp, R, vp]
    lib.sgp_apply_operator.argtypes = [vp, vp, i, i, i, vp, vp]
    lib.sgp_solver_create.argtypes = [i, ctypes.POINTER(_Problem), P, vp, vp, ctypes.POINTER(vp)]
    lib.sgp_solver_step.argtypes = [vp, i, ctypes.POINTER(i)]
    lib.sgp_solver_prepare.argtypes = [vp, i]
    lib.sgp_solver_report.argtypes = [vp, R]
    lib.sgp_solver_gradient.argtypes = [vp, vp]
    lib.sgp_solver_set_timing.argtypes = [vp, i]
    lib.sgp_solver_set_graph.argtypes = [vp, i]
    lib.sgp_solver_timing.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong), i]
    lib.sgp_solver_destroy.argtypes = [vp]
    lib.sgp_batch_deconv.argtypes = [i, ctypes.POINTER(_Problem), i, ctypes.POINTER(vp), ctypes.POINTER(vp), P,
                                     ctypes.POINTER(_Report), vp]
    lib.sgp_mosaic_deconv.argtypes = [i, vp, i, i, vp, i, f, i, i, P, vp, R, vp]
    lib.sgp_steplength_rule.argtypes = [P, i, d, d, ctypes.POINTER(d), i, d, d, d, d, ctypes.POINTER(d)]
    sz, fp = ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)
    lib.sgp_cnn_num_params.argtypes = []
    lib.sgp_cnn_create.argtypes = [fp, sz, ctypes.POINTER(vp)]
    lib.sgp_cnn_get_params.argtypes = [vp, fp, sz]
    lib.sgp_cnn_infer.argtypes = [vp, i, ctypes.POINTER(vp), fp, i, i, ctypes.POINTER(vp), vp]
    lib.sgp_cnn_loss_grad.argtypes = [vp, i, ctypes.POINTER(vp), fp, ctypes.POINTER(vp), i, i,
                                      ctypes.POINTER(d), fp, vp]
    lib.sgp_cnn_adam_step.argtypes = [vp, f, vp]
    lib.sgp_cnn_train_step.argtypes = [vp, i, ctypes.POINTER(vp), fp, ctypes.POINTER(vp), i, i, f,
                                       ctypes.POINTER(d), vp]
    lib.sgp_cnn_destroy.argtypes = [vp]
    ip = ctypes.POINTER(i)
    lib.sgp_tile_info.argtypes = [i, i, ip, ip, ip, ip]
    lib.sgp_set_tile_schedule.argtypes = [i, i, i]
    lib.sgp_get_tile_schedule.argtypes = [i, ip, ip]
    lib.sgp_save_tile_schedule.argtypes = [ctypes.c_char_p]
    lib.sgp_load_tile_schedule.argtypes = [ctypes.c_char_p]
    lib.sgp_autotune.argtypes = [ctypes.POINTER(_Problem), vp, i, ip, ip, ctypes.POINTER(d), vp]
    dp = ctypes.POINTER(d)
    lib.sgp_flux_multiplier.argtypes = [dp, dp, ctypes.c_longlong, d, i, dp, ip, ip]
    lib.sgp_strerror.restype = ctypes.c_char_p
    lib.sgp_strerror.argtypes = [i]
    lib.sgp_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("sgp_strerror", "sgp_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def default_params() -> dict:
    lib = load()
    p = _Params()
    lib.sgp_params_init(ctypes.byref(p))
    return {name: getattr(p, name) for name, _ in _Params._fields_ if name not in ("f0", "trace", "f_true")}


def _make_params(kw: dict, trace_rows: int | None, fshape=None):
    lib = load()
    p = _Params()
    lib.sgp_params_init(ctypes.byref(p))
    keep = []
    for k, v in kw.items():
        if k in ("f0", "f_true"):
            _check_dev(v, k)
            if fshape is not None:
                _check_shape(v, fshape, k)
            setattr(p, k, v.data_ptr())
            keep.append(v)
        elif k == "trace":
            continue
        elif not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        else:
            setattr(p, k, v)
    if "f0" in kw and "init" not in kw:
        p.init = INIT_USER
    trace = None
    if trace_rows:
        trace = np.zeros((trace_rows, TRACE_COLS), dtype=np.float64)
        p.trace = trace.ctypes.data
    return p, trace, keep


def _check_dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")


def _check_shape(t, shape, name):
    """The library takes every size from its integer arguments and reads or
    writes that many elements: a tensor of another shape would be accessed
    out of bounds on the device, so it is refused here."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _raise(rc):
    lib = load()
    if rc < 0:
        raise SgpError(rc, lib.sgp_last_error().decode() or lib.sgp_strerror(rc).decode())


def _report(rep: _Report, rc: int, trace):
    out = {name: getattr(rep, name) for name, _ in _Report._fields_}
    out["reason"] = REASONS.get(rep.stop_reason, str(rep.stop_reason))
    out["rc"] = rc
    if trace is not None:
        n = rep.iters + 1
        out["trace"] = {f: trace[:n, c].copy() for c, f in enumerate(TRACE_FIELDS)}
    return out


MAX_IMAGES = 8  # images per problem the library accepts (1 <= p <= 8)


def _bconst(b, p):
    if not 1 <= p <= MAX_IMAGES:
        raise ValueError(f"p = {p} images; the library takes 1..{MAX_IMAGES}")
    arr = (ctypes.c_float * MAX_IMAGES)()
    bv = np.asarray(b, dtype=np.float32).ravel() if np.ndim(b) else np.float32(b)
    if np.ndim(bv) and bv.size not in (1, p):
        raise ValueError(f"{bv.size} backgrounds given for {p} images")
    vals = np.broadcast_to(bv, (p,))
    for j in range(p):
        arr[j] = float(vals[j])
    return arr


def _solve_single(fn, g, psf, b, b_map, f, stream, trace, kw):
    import torch
    _check_dev(g, "g")
    _check_dev(psf, "psf")
    if g.dim() != 2:
        raise ValueError(f"g must be 2D [ny, nx], got shape {tuple(g.shape)}")
    ny, nx = g.shape
    _check_shape(psf, (ny, nx), "psf")
    if b_map is not None:
        _check_dev(b_map, "b_map")
        _check_shape(b_map, (ny, nx), "b_map")
    if f is None:
        f = torch.empty((ny, nx), dtype=torch.float32, device=g.device)
    _check_dev(f, "f")
    _check_shape(f, (ny, nx), "f")
    prm, tr, keep = _make_params(kw, (kw.get("max_iter", 1000) + 1) if trace else None, (ny, nx))
    rep = _Report()
    rc = fn(ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(psf.data_ptr()),
            ctypes.c_void_p(b_map.data_ptr() if b_map is not None else 0), ctypes.c_float(float(b)),
            ny, nx, ctypes.byref(prm), ctypes.c_void_p(f.data_ptr()), ctypes.byref(rep), _stream(stream))
    _raise(rc)
    return f, _report(rep, rc, tr)


def sgp_deconv(g, psf, b=0.0, *, b_map=None, f=None, stream=None, trace=False, **params):
    """SGP single-image deconvolution; returns (f, report)."""
    return _solve_single(load().sgp_deconv, g, psf, b, b_map, f, stream, trace, params)


def sgp_deconv_noalloc(g, psf, b=0.0, *, f, b_map=None, stream=None, **params):
    """sgp_deconv on the library's static device workspace (no allocation by
    the library; the caller passes f).  Returns (f, report)."""
    if "trace" in params:
        raise ValueError("sgp_deconv_noalloc keeps no trace")
    return _solve_single(load().sgp_deconv_noalloc, g, psf, b, b_map, f, stream, False, params)


def rl_deconv(g, psf, b=0.0, *, b_map=None, f=None, stream=None, trace=False, **params):
    """Richardson-Lucy single-image deconvolution (Eq. (RL); with rl_alpha != 1
    the multiplicative relaxation of Eq. (RL1); with rl_line_search=1 the
    linear relaxation of Eq. (RL2), an Armijo line search along the RL
    direction with steps up to rl_lambda_cap); returns (f, report)."""
    return _solve_single(load().rl_deconv, g, psf, b, b_map, f, stream, trace, params)


def _stack_shapes(g, psf, b_map, domain):
    """Checks a [p, ny, nx] image stack (2D for p = 1), its [p, NY, NX] PSFs
    and background maps against each other and the domain; returns the 3D
    views and (p, ny, nx, NY, NX, oy, ox)."""
    if g.dim() == 2:
        g = g.unsqueeze(0)
    if g.dim() != 3:
        raise ValueError(f"g must be [p, ny, nx] or [ny, nx], got shape {tuple(g.shape)}")
    p, ny, nx = g.shape
    if not 1 <= p <= MAX_IMAGES:
        raise ValueError(f"p = {p} images; the library takes 1..{MAX_IMAGES}")
    NY, NX, oy, ox = (int(v) for v in domain) if domain is not None else (ny, nx, 0, 0)
    if domain is not None and not (0 <= oy and 0 <= ox and oy + ny <= NY and ox + nx <= NX):
        raise ValueError(f"window {ny}x{nx} at ({oy}, {ox}) does not lie inside the {NY}x{NX} domain")
    if psf.dim() == 2 and p == 1:
        psf = psf.unsqueeze(0)
    _check_shape(psf, (p, NY, NX), "psf")
    if b_map is not None:
        _check_dev(b_map, "b_map")
        if b_map.dim() == 2 and p == 1:
            b_map = b_map.unsqueeze(0)
        _check_shape(b_map, (p, ny, nx), "b_map")
    return g, psf, b_map, (p, ny, nx, NY, NX, oy, ox)


def _solve_stack(fn, g, psf, b, b_map, f, stream, trace, kw, domain=None):
    import torch
    _check_dev(g, "g")
    _check_dev(psf, "psf")
    g, psf, b_map, (p, ny, nx, NY, NX, oy, ox) = _stack_shapes(g, psf, b_map, domain)
    if f is None:
        f = torch.empty((NY, NX), dtype=torch.float32, device=g.device)
    _check_dev(f, "f")
    _check_shape(f, (NY, NX), "f")
    prm, tr, keep = _make_params(kw, (kw.get("max_iter", 1000) + 1) if trace else None, (NY, NX))
    rep = _Report()
    bc = _bconst(b, p)
    args = [ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(psf.data_ptr()),
            ctypes.c_void_p(b_map.data_ptr() if b_map is not None else 0), ctypes.cast(bc, ctypes.c_void_p),
            p, ny, nx]
    if domain is not None:
        args += [NY, NX, oy, ox]
    rc = fn(*args, ctypes.byref(prm), ctypes.c_void_p(f.data_ptr()), ctypes.byref(rep), _stream(stream))
    _raise(rc)
    return f, _report(rep, rc, tr)


def sgp_multi_deconv(g, psf, b, *, b_map=None, f=None, stream=None, trace=False, **params):
    """SGP for p images [p, ny, nx] of one object; returns (f, report)."""
    return _solve_stack(load().sgp_multi_deconv, g, psf, b, b_map, f, stream, trace, params)


def rl_multi_deconv(g, psf, b, *, b_map=None, f=None, stream=None, trace=False, **params):
    """Multiple-image RL; returns (f, report)."""
    return _solve_stack(load().rl_multi_deconv, g, psf, b, b_map, f, stream, trace, params)


def sgp_boundary_deconv(g, psf, b, domain, *, b_map=None, f=None, stream=None, trace=False, **params):
    """SGP with boundary-effect correction; domain = (NY, NX, oy, ox)."""
    return _solve_stack(load().sgp_boundary_deconv, g, psf, b, b_map, f, stream, trace, params, domain)


def rl_boundary_deconv(g, psf, b, domain, *, b_map=None, f=None, stream=None, trace=False, **params):
    """RL with boundary-effect correction; domain = (NY, NX, oy, ox)."""
    return _solve_stack(load().rl_boundary_deconv, g, psf, b, b_map, f, stream, trace, params, domain)


def osem_deconv(g, psf, b, *, b_map=None, f=None, stream=None, trace=False, **params):
    """OSEM over the p images of g [p, ny, nx] (Algorithm 2)."""
    return _solve_stack(load().osem_deconv, g, psf, b, b_map, f, stream, trace, params)


def osem_boundary_deconv(g, psf, b, domain, *, b_map=None, f=None, stream=None, trace=False, **params):
    """OSEM with boundary-effect correction (Eq. boundaryOSEM); domain = (NY, NX, oy, ox)."""
    return _solve_stack(load().osem_boundary_deconv, g, psf, b, b_map, f, stream, trace, params, domain)


def mosaic_deconv(g, psf, b, core, margin, *, kind=KIND_SGP, f=None, stream=None, **params):
    """Mosaic of boundary-corrected subdomains: g [H, W], psf [N, N] (the FFT
    domain of every window); returns (f [H, W], report)."""
    import torch
    _check_dev(g, "g")
    _check_dev(psf, "psf")
    if g.dim() != 2:
        raise ValueError(f"g must be 2D [H, W], got shape {tuple(g.shape)}")
    H, W = g.shape
    N = psf.shape[-1]
    if psf.shape != (N, N):
        raise ValueError("psf must be N x N")
    if f is None:
        f = torch.empty_like(g)
    _check_dev(f, "f")
    _check_shape(f, (H, W), "f")
    prm, _, _ = _make_params(params, None)
    rep = _Report()
    rc = load().sgp_mosaic_deconv(int(kind), ctypes.c_void_p(g.data_ptr()), H, W, ctypes.c_void_p(psf.data_ptr()),
                                  N, ctypes.c_float(float(b)), int(core), int(margin), ctypes.byref(prm),
                                  ctypes.c_void_p(f.data_ptr()), ctypes.byref(rep), _stream(stream))
    _raise(rc)
    return f, _report(rep, rc, None)


def apply_operator(psf, x, adjoint=False, out=None, stream=None):
    """out = A x (or A^T x) for the periodic operator of a unit-volume PSF."""
    import torch
    _check_dev(psf, "psf")
    _check_dev(x, "x")
    if x.dim() != 2:
        raise ValueError(f"x must be 2D [ny, nx], got shape {tuple(x.shape)}")
    ny, nx = x.shape
    _check_shape(psf, (ny, nx), "psf")
    if out is None:
        out = torch.empty_like(x)
    _check_dev(out, "out")
    _check_shape(out, (ny, nx), "out")
    rc = load().sgp_apply_operator(ctypes.c_void_p(psf.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   ny, nx, 1 if adjoint else 0, ctypes.c_void_p(out.data_ptr()),
                                   _stream(stream))
    _raise(rc)
    return out


def release_cache():
    return load().sgp_release_cache()


TILE_VARIANTS = 4  # per length: bit 0 the workgroup shape, bit 1 the transform plan


def tile_info(L, variant):
    """Workgroup shape of tile variant ``variant`` (0..3) at FFT length L (no
    GPU needed): row-kernel threads and row pairs, column-kernel threads and
    columns; the points per thread of its transforms are L * row_pairs /
    row_threads."""
    lib = load()
    v = [ctypes.c_int() for _ in range(4)]
    _raise(lib.sgp_tile_info(int(L), int(variant), *[ctypes.byref(x) for x in v]))
    return dict(row_threads=v[0].value, row_pairs=v[1].value, col_threads=v[2].value, col_width=v[3].value)


def set_tile_schedule(L, row_variant, col_variant):
    _raise(load().sgp_set_tile_schedule(int(L), int(row_variant), int(col_variant)))


def get_tile_schedule(L):
    r, c = ctypes.c_int(), ctypes.c_int()
    _raise(load().sgp_get_tile_schedule(int(L), ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def save_tile_schedule(path):
    _raise(load().sgp_save_tile_schedule(os.fsencode(path)))


def load_tile_schedule(path):
    _raise(load().sgp_load_tile_schedule(os.fsencode(path)))


def autotune(g, psf, b, *, domain=None, iters=20, stream=None):
    """Times every distinct tile combination on this problem (``g``/``psf``
    as for Solver) and keeps the fastest in the schedule table.  Variants
    0..3: bit 0 the workgroup shape, bit 1 the transform plan.  Returns
    (row_variant, col_variant, ms) with ms[(r, c)] the least ms per
    iteration over the timed runs (absent for a combination equal to
    another)."""
    import torch
    lib = load()
    _check_dev(g, "g")
    _check_dev(psf, "psf")
    g3, psf3, _, (p, ny, nx, NY, NX, oy, ox) = _stack_shapes(g, psf, None, domain)
    bc = _bconst(b, p)
    pr = _Problem(g3.data_ptr(), psf3.data_ptr(), None, ctypes.cast(bc, ctypes.c_void_p), p, ny, nx, NY, NX,
                  oy, ox, 1 if domain is not None else 0)
    f = torch.empty((NY, NX), dtype=torch.float32, device=g.device)
    r, c = ctypes.c_int(), ctypes.c_int()
    ms = (ctypes.c_double * (TILE_VARIANTS * TILE_VARIANTS))()
    _raise(lib.sgp_autotune(ctypes.byref(pr), ctypes.c_void_p(f.data_ptr()), int(iters), ctypes.byref(r),
                            ctypes.byref(c), ms, _stream(stream)))
    times = {(k // TILE_VARIANTS, k % TILE_VARIANTS): ms[k] for k in range(TILE_VARIANTS * TILE_VARIANTS)
             if ms[k] >= 0}
    return r.value, c.value, times


class Solver:
    """Stepping solver (sgp_solver_* of the C ABI).  ``g``/``psf`` are
    [p, ny, nx] / [p, NY, NX] (or 2D) CUDA tensors; ``domain`` = (NY, NX, oy,
    ox) selects boundary-effect correction.  The tensors must stay alive while
    the solver exists; ``f`` is updated in place."""

    def __init__(self, kind, g, psf, b, *, domain=None, b_map=None, f=None, stream=None,
                 trace=False, **params):
        import torch
        lib = load()
        _check_dev(g, "g")
        _check_dev(psf, "psf")
        g3, psf3, b_map, (p, ny, nx, NY, NX, oy, ox) = _stack_shapes(g, psf, b_map, domain)
        if f is None:
            f = torch.empty((NY, NX), dtype=torch.float32, device=g.device)
        _check_dev(f, "f")
        _check_shape(f, (NY, NX), "f")
        self._bc = _bconst(b, p)
        pr = _Problem(g3.data_ptr(), psf3.data_ptr(), b_map.data_ptr() if b_map is not None else None,
                      ctypes.cast(self._bc, ctypes.c_void_p), p, ny, nx, NY, NX, oy, ox,
                      1 if domain is not None else 0)
        self._prm, self._trace, self._keep = _make_params(
            params, (params.get("max_iter", 1000) + 1) if trace else None, (NY, NX))
        self._keep += [g3, psf3, b_map, f]
        self.f = f
        self._h = ctypes.c_void_p()
        rc = lib.sgp_solver_create(kind, ctypes.byref(pr), ctypes.byref(self._prm),
                                   ctypes.c_void_p(f.data_ptr()), _stream(stream), ctypes.byref(self._h))
        _raise(rc)

    def step(self, n):
        done = ctypes.c_int(0)
        _raise(load().sgp_solver_step(self._h, int(n), ctypes.byref(done)))
        return bool(done.value)

    def prepare(self, n):
        """Captures the graphs a later step(n) replays (no iteration runs)."""
        _raise(load().sgp_solver_prepare(self._h, int(n)))

    def report(self):
        rep = _Report()
        rc = load().sgp_solver_report(self._h, ctypes.byref(rep))
        _raise(rc)
        return _report(rep, rc, self._trace)

    def gradient(self):
        """The gradient the SGP solver carries at its current iterate
        (a new [NY, NX] tensor)."""
        import torch
        out = torch.empty_like(self.f)
        _raise(load().sgp_solver_gradient(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_timing(self, on=True):
        _raise(load().sgp_solver_set_timing(self._h, 1 if on else 0))

    def set_graph(self, on=True):
        _raise(load().sgp_solver_set_graph(self._h, 1 if on else 0))

    def timing(self):
        n = len(KCLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        _raise(load().sgp_solver_timing(self._h, ms, cnt, n))
        return {KCLASSES[i]: (ms[i], cnt[i]) for i in range(n)}

    def close(self):
        if self._h:
            load().sgp_solver_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def steplength_rule(k, alpha, tau, Q, a, c1, c2, e, **params):
    """The device steplength rule (Sect. 2.1) evaluated on the host."""
    prm, _, _ = _make_params(params, None)
    q = (ctypes.c_double * 8)(*list(Q)[:8])
    out = (ctypes.c_double * 16)()
    rc = load().sgp_steplength_rule(ctypes.byref(prm), int(k), float(alpha), float(tau), q, len(Q),
                                    float(a), float(c1), float(c2), float(e), out)
    _raise(rc)
    nq = int(out[7])
    return dict(a1=out[0], a2=out[1], alpha_next=out[2], tau=out[3], alt=int(out[4]),
                br1=int(out[5]), br2=int(out[6]), Q=[out[8 + i] for i in range(nq)])


def flux_multiplier(z, D, c, max_steps=8):
    """The device's search for the flux-projection multiplier run on the host
    (validation): returns (mu, Newton steps, converged, return code)."""
    z = np.ascontiguousarray(z, dtype=np.float64).ravel()
    D = np.ascontiguousarray(D, dtype=np.float64).ravel()
    if z.size != D.size:
        raise ValueError("z and D must have the same size")
    mu, steps, conv = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = load().sgp_flux_multiplier(z.ctypes.data_as(dp), D.ctypes.data_as(dp), z.size, float(c), int(max_steps),
                                    ctypes.byref(mu), ctypes.byref(steps), ctypes.byref(conv))
    _raise(rc)
    return mu.value, steps.value, bool(conv.value), rc


def batch_deconv(gs, psfs, bs, *, kind=KIND_SGP, f0s=None, fs=None, domains=None, stream=None, **params):
    """Many single-image problems (uneven sizes) in one batched run.
    gs, psfs: lists of 2D CUDA tensors; bs: constant backgrounds; f0s: optional
    starts (init=INIT_USER or INIT_WARM); domains: optional list with, per
    problem, None (periodic) or (NY, NX, oy, ox) for boundary-effect
    correction (its PSF, f and f0 are then NY x NX).  Returns (list of f,
    list of reports)."""
    import torch
    lib = load()
    n = len(gs)
    if len(psfs) != n or len(bs) != n or any(x is not None and len(x) != n for x in (fs, f0s, domains)):
        raise ValueError("gs, psfs, bs (and fs, f0s, domains when given) must have one entry per problem")
    doms = [None] * n if domains is None else [None if d is None else tuple(int(v) for v in d) for d in domains]
    if fs is None:
        fs = [torch.empty((d[0], d[1]) if d else tuple(g.shape), dtype=torch.float32, device=g.device)
              for g, d in zip(gs, doms)]
    probs = (_Problem * n)()
    keep = [gs, psfs, fs, f0s]
    bcs = []
    for i in range(n):
        _check_dev(gs[i], "g")
        _check_dev(psfs[i], "psf")
        _check_dev(fs[i], "f")
        if gs[i].dim() != 2:
            raise ValueError(f"g[{i}] must be 2D [ny, nx], got shape {tuple(gs[i].shape)}")
        ny, nx = gs[i].shape
        NY, NX, oy, ox = doms[i] if doms[i] else (ny, nx, 0, 0)
        if doms[i] and not (0 <= oy and 0 <= ox and oy + ny <= NY and ox + nx <= NX):
            raise ValueError(f"problem {i}: window {ny}x{nx} at ({oy}, {ox}) outside the {NY}x{NX} domain")
        _check_shape(psfs[i], (NY, NX), f"psf[{i}]")
        _check_shape(fs[i], (NY, NX), f"f[{i}]")
        if f0s is not None:
            _check_shape(f0s[i], (NY, NX), f"f0[{i}]")
        bc = (ctypes.c_float * 1)(float(bs[i]))
        bcs.append(bc)
        probs[i] = _Problem(gs[i].data_ptr(), psfs[i].data_ptr(), None, ctypes.cast(bc, ctypes.c_void_p),
                            1, ny, nx, NY, NX, oy, ox, 1 if doms[i] else 0)
    fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    f0p = None
    if f0s is not None:
        for t in f0s:
            _check_dev(t, "f0")
        f0p = (ctypes.c_void_p * n)(*[t.data_ptr() for t in f0s])
        if "init" not in params:
            params["init"] = INIT_USER
    prm, _, _ = _make_params(params, None)
    if f0s is not None:
        prm.f0 = f0s[0].data_ptr()
    reps = (_Report * n)()
    rc = lib.sgp_batch_deconv(kind, probs, n, fp, f0p, ctypes.byref(prm), reps, _stream(stream))
    _raise(rc)
    return fs, [_report(reps[i], rc, None) for i in range(n)]


# ------------------------------------------------------------------ warm-start network
def _ptrs(ts, name):
    for t in ts:
        _check_dev(t, name)
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


class CnnNet:
    """Handle of the warm-start network (sgp_cnn_* of the C ABI).  ``params``
    is the float32 parameter vector (include/sgpcnn.h gives its layout)."""

    def __init__(self, params):
        lib = load()
        self.n_params = lib.sgp_cnn_num_params()
        theta = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if theta.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {theta.size}")
        self._h = ctypes.c_void_p()
        _raise(lib.sgp_cnn_create(theta.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), theta.size,
                                  ctypes.byref(self._h)))

    @staticmethod
    def _shape(gs):
        shapes = {tuple(g.shape) for g in gs}
        if len(shapes) != 1 or len(next(iter(shapes))) != 2:
            raise ValueError("one call takes 2D images of one shape")
        return next(iter(shapes))

    @staticmethod
    def _same(gs, others, name):
        if len(others) != len(gs):
            raise ValueError(f"{len(others)} {name} tensors for {len(gs)} images")
        for i, t in enumerate(others):
            _check_shape(t, gs[0].shape, f"{name}[{i}]")

    @staticmethod
    def _backgrounds(bs, n):
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(bs, dtype=np.float32).ravel(), (n,)))
        return b

    def params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _raise(load().sgp_cnn_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         out.size))
        return out

    def infer(self, gs, bs, out=None, stream=None):
        """Start images for images of one shape; returns a list of tensors."""
        import torch
        ny, nx = self._shape(gs)
        if out is None:
            out = [torch.empty_like(g) for g in gs]
        self._same(gs, out, "f0")
        b = self._backgrounds(bs, len(gs))
        _raise(load().sgp_cnn_infer(self._h, len(gs), _ptrs(gs, "g"),
                                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ny, nx,
                                    _ptrs(out, "f0"), _stream(stream)))
        return out

    def loss_grad(self, gs, bs, targets, stream=None):
        """(mean loss, gradient as float32 numpy) of one batch."""
        ny, nx = self._shape(gs)
        self._same(gs, targets, "target")
        b = self._backgrounds(bs, len(gs))
        loss = ctypes.c_double()
        grad = np.empty(self.n_params, dtype=np.float32)
        _raise(load().sgp_cnn_loss_grad(self._h, len(gs), _ptrs(gs, "g"),
                                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _ptrs(targets, "target"),
                                        ny, nx, ctypes.byref(loss),
                                        grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
        return loss.value, grad

    def adam_step(self, lr, stream=None):
        _raise(load().sgp_cnn_adam_step(self._h, float(lr), _stream(stream)))

    def train_step(self, gs, bs, targets, lr, stream=None):
        """Loss, gradient and Adam step on one batch; returns the loss."""
        ny, nx = self._shape(gs)
        self._same(gs, targets, "target")
        b = self._backgrounds(bs, len(gs))
        loss = ctypes.c_double()
        _raise(load().sgp_cnn_train_step(self._h, len(gs), _ptrs(gs, "g"),
                                         b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         _ptrs(targets, "target"), ny, nx, float(lr), ctypes.byref(loss),
                                         _stream(stream)))
        return loss.value

    def close(self):
        if self._h:
            load().sgp_cnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
