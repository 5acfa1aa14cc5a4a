"""ctypes binding of libsgn (include/sgn.h).

Argument marshalling only: every step of the solver runs in the HIP
library.  PyTorch supplies device memory (the fields and the workspace) and
the stream.  The library must have been built (python -m
paper_2306_09731_amd.build); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsgn.so")

SGN_OK = 0
SGN_ERR_INVALID_ARG = 1
SGN_ERR_UNSUPPORTED = 2
SGN_ERR_HIP = 3
SGN_ERR_NOT_CONVERGED = 4
SGN_ERR_CAVITATION = 5
SGN_ERR_NONFINITE = 6
SGN_FP64 = 0
SGN_FP32_MIXED = 1
SGN_GUESS_PREVIOUS = 0
SGN_GUESS_STAGE_INCREMENT = 1
SGN_KERNEL_ROW_MATVEC = 0
SGN_KERNEL_COL_BASIS = 1
SGN_KERNEL_COL_PRECOND_DOT = 2
SGN_KERNEL_GS_UPDATE = 3
SGN_KERNEL_ROW_FLUX = 4
SGN_KERNEL_COL_FLUX = 5
SGN_CNN_LAYERS = 6
SGN_CNN_CH = 32
SGN_CNN_PARAMS = SGN_CNN_LAYERS * (9 * SGN_CNN_CH * SGN_CNN_CH + SGN_CNN_CH)
KERNEL_NAMES = {0: "row_matvec", 1: "col_basis", 2: "col_precond_dot", 3: "gs_update", 4: "row_flux",
                5: "col_flux"}


class sgn_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
        ("g", ctypes.c_double), ("h_inf", ctypes.c_double),
        ("precision", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
        ("gmres_tol", ctypes.c_double),
        ("gmres_max_iters", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("krasny", ctypes.c_double),
        ("invariants_tol", ctypes.c_double),
        ("dealias", ctypes.c_int32), ("guess", ctypes.c_int32),
    ]


class sgn_solve_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("converged", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("rel_resid_precond", ctypes.c_double), ("rel_resid_true", ctypes.c_double),
    ]


class sgn_refine_info(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("rel_resid_first", ctypes.c_double), ("rel_resid_true", ctypes.c_double)]


class sgn_fgmres_info(ctypes.Structure):
    _fields_ = [("fgmres_iters", ctypes.c_int32), ("fgmres_cycles", ctypes.c_int32),
                ("gmres_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("fgmres_rel_resid", ctypes.c_double), ("rel_resid_true", ctypes.c_double)]


class sgn_refined_step_info(ctypes.Structure):
    _fields_ = [("inner_iters", ctypes.c_int64), ("rounds", ctypes.c_int64), ("solves", ctypes.c_int32),
                ("max_rounds_per_solve", ctypes.c_int32), ("max_rel_resid", ctypes.c_double),
                ("min_h", ctypes.c_double)]


class sgn_step_info(ctypes.Structure):
    _fields_ = [
        ("total_iters", ctypes.c_int64), ("max_iters_per_solve", ctypes.c_int32),
        ("solves", ctypes.c_int32), ("min_h", ctypes.c_double),
        ("any_unconverged", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]


class sgn_invariants_out(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("px", ctypes.c_double), ("py", ctypes.c_double),
        ("energy", ctypes.c_double), ("min_h", ctypes.c_double), ("max_h", ctypes.c_double),
        ("curl_l2", ctypes.c_double), ("spectral_tail", ctypes.c_double),
    ]


_VP = ctypes.c_void_p
_ENSEMBLE_ARGS = [ctypes.c_int32, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                  ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.POINTER(sgn_step_info)]

_SIGNATURES = {
    "sgn_config_default": (None, [ctypes.POINTER(sgn_config), ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_double]),
    "sgn_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(sgn_config)]),
    "sgn_init": (ctypes.c_int, [ctypes.POINTER(sgn_config), _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "sgn_destroy": (ctypes.c_int, [_VP]),
    "sgn_elliptic_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(sgn_solve_info)]),
    "sgn_rhs": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(sgn_solve_info)]),
    "sgn_launch_shape": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "sgn_elliptic_solve_refined": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32,
                                                  ctypes.POINTER(sgn_refine_info)]),
    "sgn_rk4_step_refined": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_int32, ctypes.POINTER(sgn_refined_step_info)]),
    "sgn_rk4_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(sgn_step_info)]),
    "sgn_rk4_step_graph": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(sgn_step_info),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "sgn_invariants": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(sgn_invariants_out)]),
    "sgn_derivative": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP]),
    "sgn_apply_operator": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32]),
    "sgn_apply_precond": (ctypes.c_int, [_VP, _VP, _VP]),
    "sgn_apply_operator_noalloc": (ctypes.c_int, [ctypes.POINTER(sgn_config), _VP, _VP, _VP, ctypes.c_int32, _VP]),
    "sgn_krasny_filter": (ctypes.c_int, [_VP, _VP]),
    "sgn_rk4_step_ensemble": (ctypes.c_int, _ENSEMBLE_ARGS),
    "sgn_rk4_step_ensemble_graph": (ctypes.c_int, _ENSEMBLE_ARGS),
    "sgn_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "sgn_kernel_timing": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "sgn_kernel_time": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "sgn_cnn_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "sgn_cnn_init": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "sgn_cnn_destroy": (ctypes.c_int, [_VP]),
    "sgn_cnn_set_params": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float)]),
    "sgn_cnn_get_params": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float)]),
    "sgn_cnn_forward": (ctypes.c_int, [_VP, _VP, _VP]),
    "sgn_cnn_gradients": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_double)]),
    "sgn_cnn_train_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
    "sgn_cnn_last_error": (ctypes.c_char_p, [_VP]),
    "sgn_learned_guess_attach": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32]),
    "sgn_learned_guess_recorded": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "sgn_learned_guess_stages": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "sgn_elliptic_solve_fgmres": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32,
                                                 ctypes.POINTER(sgn_fgmres_info)]),
    "sgn_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sgn_last_error": (ctypes.c_char_p, [_VP]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsgn.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -m paper_2306_09731_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SgnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def config_default(nx: int, ny: int, Lx: float, Ly: float, **overrides) -> sgn_config:
    lib = load_library()
    cfg = sgn_config()
    lib.sgn_config_default(ctypes.byref(cfg), nx, ny, Lx, Ly)
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def sgn_workspace_bytes(cfg: sgn_config) -> int:
    return int(load_library().sgn_workspace_bytes(ctypes.byref(cfg)))


@dataclasses.dataclass
class Context:
    handle: ctypes.c_void_p
    cfg: sgn_config
    workspace: object  # torch.Tensor (uint8, device)
    device: object

    def last_error(self) -> str:
        msg = load_library().sgn_last_error(self.handle)
        return msg.decode() if msg else ""

    def close(self):
        if self.handle:
            load_library().sgn_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def _check(ctx: Context | None, status: int, allow=(SGN_OK,)):
    if status in allow:
        return status
    lib = load_library()
    msg = lib.sgn_status_string(status).decode()
    if ctx is not None:
        extra = ctx.last_error()
        if extra:
            msg = f"{msg}: {extra}"
    raise SgnError(status, msg)


def field_dtype(cfg: sgn_config):
    """torch dtype of the fields for this configuration's precision."""
    import torch
    return torch.float32 if cfg.precision == SGN_FP32_MIXED else torch.float64


def _field(ctx: Context, t, name: str):
    import torch
    cfg = ctx.cfg
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    dt = field_dtype(cfg)
    shape = (cfg.ny, cfg.nx) if cfg.batch == 1 else (cfg.batch, cfg.ny, cfg.nx)
    if t.dtype != dt or not t.is_contiguous() or t.device != ctx.device or tuple(t.shape) != shape:
        raise ValueError(f"{name} must be a contiguous {dt} tensor of shape {shape} on {ctx.device}")
    return ctypes.c_void_p(t.data_ptr())


def _infos(ctx: Context, cls):
    """One info struct per ensemble member."""
    return (cls * max(ctx.cfg.batch, 1))()


def _one_or_list(ctx: Context, arr):
    return arr[0] if ctx.cfg.batch == 1 else [arr[i] for i in range(ctx.cfg.batch)]


def sgn_init(cfg: sgn_config, device="cuda:0", stream=None) -> Context:
    """Allocate the workspace as a torch tensor and initialise a context on the
    given (or current) torch stream."""
    import torch
    lib = load_library()
    device = torch.device(device)
    nbytes = sgn_workspace_bytes(cfg)
    if nbytes == 0:
        raise SgnError(SGN_ERR_INVALID_ARG, "invalid configuration")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    ws_view = ws[off:off + nbytes]
    if stream is None:
        stream = torch.cuda.current_stream(device)
    handle = ctypes.c_void_p()
    st = lib.sgn_init(ctypes.byref(cfg), ctypes.c_void_p(ws_view.data_ptr()), nbytes,
                      ctypes.c_void_p(stream.cuda_stream), ctypes.byref(handle))
    _check(None, st)
    return Context(handle=handle, cfg=cfg, workspace=ws, device=device)


def sgn_elliptic_solve(ctx: Context, h, b, sigma):
    """Solve L_h sigma = b (sigma: initial guess in, solution out).  Returns the
    sgn_solve_info, or one per member for an ensemble context."""
    info = _infos(ctx, sgn_solve_info)
    st = load_library().sgn_elliptic_solve(ctx.handle, _field(ctx, h, "h"), _field(ctx, b, "b"),
                                           _field(ctx, sigma, "sigma"), info)
    _check(ctx, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return _one_or_list(ctx, info)


def sgn_rhs(ctx: Context, h, vx, vy, sigma, dh, dvx, dvy):
    info = _infos(ctx, sgn_solve_info)
    st = load_library().sgn_rhs(ctx.handle, _field(ctx, h, "h"), _field(ctx, vx, "vx"), _field(ctx, vy, "vy"),
                                _field(ctx, sigma, "sigma"), _field(ctx, dh, "dh"), _field(ctx, dvx, "dvx"),
                                _field(ctx, dvy, "dvy"), info)
    _check(ctx, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return _one_or_list(ctx, info)


def sgn_launch_shape(ctx: Context) -> dict:
    """The context's Arnoldi schedule, tile targets and resulting block shapes."""
    out = (ctypes.c_int32 * 8)()
    _check(ctx, load_library().sgn_launch_shape(ctx.handle, out))
    keys = ("arnoldi", "tile_blocks", "row_threads", "row_pairs_per_block", "row_pairs_per_block3",
            "cols_per_tile", "cols_per_tile2", "row_radix")
    return dict(zip(keys, list(out)))


def sgn_elliptic_solve_refined(ctx64: Context, ctx32: Context, h, b, sigma, tol: float,
                               max_rounds: int = 8) -> sgn_refine_info:
    """FP64 solution by FP32 corrections (FP64 fields h, b, sigma of ctx64's grid)."""
    info = sgn_refine_info()
    st = load_library().sgn_elliptic_solve_refined(ctx64.handle, ctx32.handle, _field(ctx64, h, "h"),
                                                   _field(ctx64, b, "b"), _field(ctx64, sigma, "sigma"), float(tol),
                                                   int(max_rounds), ctypes.byref(info))
    _check(ctx64, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return info


def sgn_rk4_step(ctx: Context, h, vx, vy, sigma, dt: float, nsteps: int = 1):
    """nsteps RK4 steps in place.  Returns the sgn_step_info, or one per member
    for an ensemble context."""
    info = _infos(ctx, sgn_step_info)
    st = load_library().sgn_rk4_step(ctx.handle, _field(ctx, h, "h"), _field(ctx, vx, "vx"),
                                     _field(ctx, vy, "vy"), _field(ctx, sigma, "sigma"), float(dt),
                                     int(nsteps), info)
    _check(ctx, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return _one_or_list(ctx, info)


def sgn_rk4_step_refined(ctx64: Context, ctx32: Context, h, vx, vy, sigma, dt: float, nsteps: int = 1,
                         tol: float = 1e-10, max_rounds: int = 8) -> sgn_refined_step_info:
    """FP64 RK4 steps whose stage solves are FP32-corrected refinements (FP64 fields of ctx64's grid)."""
    info = sgn_refined_step_info()
    st = load_library().sgn_rk4_step_refined(ctx64.handle, ctx32.handle, _field(ctx64, h, "h"),
                                             _field(ctx64, vx, "vx"), _field(ctx64, vy, "vy"),
                                             _field(ctx64, sigma, "sigma"), float(dt), int(nsteps), float(tol),
                                             int(max_rounds), ctypes.byref(info))
    _check(ctx64, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return info


def sgn_rk4_step_graph(ctx: Context, h, vx, vy, sigma, dt: float, nsteps: int = 1, iter_budget: int = 0):
    """sgn_rk4_step with every step replayed as one captured HIP graph.
    Returns (sgn_step_info, number of steps run as graph replays)."""
    info = sgn_step_info()
    rep = ctypes.c_int32(0)
    st = load_library().sgn_rk4_step_graph(ctx.handle, _field(ctx, h, "h"), _field(ctx, vx, "vx"),
                                           _field(ctx, vy, "vy"), _field(ctx, sigma, "sigma"), float(dt),
                                           int(nsteps), int(iter_budget), ctypes.byref(info), ctypes.byref(rep))
    _check(ctx, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return info, int(rep.value)


def sgn_rk4_step_ensemble(ctxs, fields, dts, nsteps: int, graphs: bool = False):
    """nsteps RK4 steps of every context; fields[i] = (h, vx, vy, sigma) of
    context i ([batch][ny][nx] for a context of several members), dts[i] its
    step; graphs: each context's steps as captured-graph replays (single-grid
    contexts only).  Returns the list of sgn_step_info, one per member, the
    contexts' members in order."""
    n = len(ctxs)
    if not (len(fields) == n and len(dts) == n):
        raise ValueError("one field tuple and one dt per context")
    arr = lambda vals: (_VP * max(n, 1))(*vals)
    ptrs = [[_field(c, f[k], name) for c, f in zip(ctxs, fields)] for k, name in enumerate(("h", "vx", "vy", "sigma"))]
    total = sum(c.cfg.batch for c in ctxs)
    infos = (sgn_step_info * max(total, 1))()
    lib = load_library()
    fn = lib.sgn_rk4_step_ensemble_graph if graphs else lib.sgn_rk4_step_ensemble
    st = fn(n, arr([c.handle for c in ctxs]), *(arr(p) for p in ptrs), (ctypes.c_double * max(n, 1))(*dts), nsteps,
            infos)
    _check(None, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return [infos[i] for i in range(total)]


ARNOLDI_SCHEDULES = {0: "four kernels, one chain", 1: "four kernels, two chains", 2: "three kernels"}


def sgn_autotune(ctx: Context) -> int:
    """Pick and keep the fastest Arnoldi kernel schedule for this context."""
    chosen = ctypes.c_int32()
    _check(ctx, load_library().sgn_autotune(ctx.handle, ctypes.byref(chosen)))
    return chosen.value


def sgn_invariants(ctx: Context, h, vx, vy, sigma):
    """Invariants as a dict, or a list of dicts (one per member) for an ensemble context."""
    out = _infos(ctx, sgn_invariants_out)
    st = load_library().sgn_invariants(ctx.handle, _field(ctx, h, "h"), _field(ctx, vx, "vx"),
                                       _field(ctx, vy, "vy"), _field(ctx, sigma, "sigma"), out)
    _check(ctx, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    d = [{name: getattr(o, name) for name, _ in sgn_invariants_out._fields_} for o in out]
    return d[0] if ctx.cfg.batch == 1 else d


def sgn_derivative(ctx: Context, axis: int, f, out):
    _check(ctx, load_library().sgn_derivative(ctx.handle, int(axis), _field(ctx, f, "f"), _field(ctx, out, "out")))


def sgn_apply_operator(ctx: Context, h, s, out, precondition: bool = False):
    _check(ctx, load_library().sgn_apply_operator(ctx.handle, _field(ctx, h, "h"), _field(ctx, s, "s"),
                                                  _field(ctx, out, "out"), 1 if precondition else 0))


SGN_NOALLOC_MAX_POINTS = 1 << 20


def sgn_apply_operator_noalloc(cfg: sgn_config, h, s, out, precondition: bool = False, stream=None):
    """sgn_apply_operator without a context: the library's fixed device
    scratch instead of a workspace (nothing is allocated).  Enqueued on the
    given (or the tensors' current) stream; does not synchronise."""
    import torch
    device = h.device if isinstance(h, torch.Tensor) else None
    view = Context(handle=None, cfg=cfg, workspace=None, device=device)
    args = [_field(view, t, name) for t, name in ((h, "h"), (s, "s"), (out, "out"))]
    if stream is None:
        stream = torch.cuda.current_stream(device)
    st = load_library().sgn_apply_operator_noalloc(ctypes.byref(cfg), *args, 1 if precondition else 0,
                                                   ctypes.c_void_p(stream.cuda_stream))
    if st != SGN_OK:
        lib = load_library()
        raise SgnError(st, f"{lib.sgn_status_string(st).decode()}: {lib.sgn_last_error(None).decode()}")


def sgn_apply_precond(ctx: Context, r, out):
    _check(ctx, load_library().sgn_apply_precond(ctx.handle, _field(ctx, r, "r"), _field(ctx, out, "out")))


def sgn_krasny_filter(ctx: Context, f):
    _check(ctx, load_library().sgn_krasny_filter(ctx.handle, _field(ctx, f, "f")))


def sgn_kernel_timing(ctx: Context, kind: int, enable: bool, period: int = 1):
    """Start (events on every period-th launch of the class) or stop timing."""
    _check(ctx, load_library().sgn_kernel_timing(ctx.handle, int(kind), int(period) if enable else 0))


def sgn_kernel_time(ctx: Context, kind: int):
    """(launches, total_ms, algo_bytes) of the timed kernel class since timing
    was enabled; algo_bytes counts the launches that did work."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    b = ctypes.c_double()
    _check(ctx, load_library().sgn_kernel_time(ctx.handle, int(kind), ctypes.byref(n), ctypes.byref(ms),
                                               ctypes.byref(b)))
    return int(n.value), float(ms.value), float(b.value)


# ---- learned initial guess (network context) ------------------------------

@dataclasses.dataclass
class CnnContext:
    handle: ctypes.c_void_p
    H: int
    W: int
    workspace: object
    device: object

    def last_error(self) -> str:
        msg = load_library().sgn_cnn_last_error(self.handle)
        return msg.decode() if msg else ""

    def close(self):
        if self.handle:
            load_library().sgn_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def _cnn_check(net, status, allow=(SGN_OK,)):
    if status in allow:
        return status
    msg = load_library().sgn_status_string(status).decode()
    extra = net.last_error() if net is not None else ""
    raise SgnError(status, f"{msg}: {extra}" if extra else msg)


def cnn_workspace_bytes(H: int, W: int) -> int:
    return int(load_library().sgn_cnn_workspace_bytes(H, W))


def cnn_init(H: int, W: int, device="cuda:0", stream=None) -> CnnContext:
    import torch
    lib = load_library()
    device = torch.device(device)
    nbytes = cnn_workspace_bytes(H, W)
    if nbytes == 0:
        raise SgnError(SGN_ERR_UNSUPPORTED, f"unsupported network grid {H}x{W}")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    if stream is None:
        stream = torch.cuda.current_stream(device)
    handle = ctypes.c_void_p()
    st = lib.sgn_cnn_init(H, W, ctypes.c_void_p(ws.data_ptr() + off), nbytes, ctypes.c_void_p(stream.cuda_stream),
                          ctypes.byref(handle))
    _cnn_check(None, st)
    return CnnContext(handle=handle, H=H, W=W, workspace=ws, device=device)


def _f32_array(a, n):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def cnn_set_params(net: CnnContext, params):
    a = _f32_array(params, SGN_CNN_PARAMS)
    _cnn_check(net, load_library().sgn_cnn_set_params(net.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def cnn_get_params(net: CnnContext):
    import numpy as np
    a = np.empty(SGN_CNN_PARAMS, dtype=np.float32)
    _cnn_check(net, load_library().sgn_cnn_get_params(net.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return a


def _cnn_field(net: CnnContext, t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            and tuple(t.shape) == shape):
        raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor of shape {shape}")
    return ctypes.c_void_p(t.data_ptr())


def cnn_forward(net: CnnContext, in3, out):
    _cnn_check(net, load_library().sgn_cnn_forward(net.handle, _cnn_field(net, in3, (net.H, net.W, 3), "in3"),
                                                   _cnn_field(net, out, (net.H, net.W), "out")))


def cnn_gradients(net: CnnContext, in3, target):
    """(gradients as a float32 array of SGN_CNN_PARAMS values, loss)."""
    import numpy as np
    g = np.empty(SGN_CNN_PARAMS, dtype=np.float32)
    loss = ctypes.c_double()
    _cnn_check(net, load_library().sgn_cnn_gradients(
        net.handle, _cnn_field(net, in3, (net.H, net.W, 3), "in3"), _cnn_field(net, target, (net.H, net.W), "target"),
        g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
    return g, loss.value


def cnn_train_step(net: CnnContext, in3, target, lr: float) -> float:
    loss = ctypes.c_double()
    _cnn_check(net, load_library().sgn_cnn_train_step(
        net.handle, _cnn_field(net, in3, (net.H, net.W, 3), "in3"), _cnn_field(net, target, (net.H, net.W), "target"),
        float(lr), ctypes.byref(loss)))
    return loss.value


def learned_guess_attach(ctx: Context, net: CnnContext | None = None, record=None):
    """Attach a network (or None) and a recorder: record is a float32 CUDA tensor
    of shape (capacity, 4, H, W) (input channels as [H][W][3] then the target),
    or None."""
    import torch
    cap, ptr = 0, None
    if record is not None:
        H, W = ctx.cfg.ny, ctx.cfg.nx
        if not (isinstance(record, torch.Tensor) and record.is_cuda and record.dtype == torch.float32
                and record.is_contiguous() and record.dim() == 4 and tuple(record.shape[1:]) == (4, H, W)):
            raise ValueError(f"record: expected a contiguous float32 CUDA tensor of shape (capacity, 4, {H}, {W})")
        cap, ptr = record.shape[0], ctypes.c_void_p(record.data_ptr())
    _check(ctx, load_library().sgn_learned_guess_attach(ctx.handle, net.handle if net is not None else None, ptr, cap))
    ctx.learned = (net, record)  # keep both alive while attached


def learned_guess_recorded(ctx: Context) -> int:
    n = ctypes.c_int64()
    _check(ctx, load_library().sgn_learned_guess_recorded(ctx.handle, ctypes.byref(n)))
    return n.value


def learned_guess_stages(ctx: Context, stage_mask: int):
    """RK stages whose solves the attached network corrects (bit s: stage s;
    0xF every stage, 0x1 once per step)."""
    _check(ctx, load_library().sgn_learned_guess_stages(ctx.handle, int(stage_mask)))


def sgn_elliptic_solve_fgmres(ctx: Context, net: CnnContext, h, b, sigma, max_iters: int = 40) -> sgn_fgmres_info:
    """Flexible GMRES with the network as right preconditioner, then plain
    GMRES from its result (sigma: initial guess in, solution out)."""
    info = sgn_fgmres_info()
    st = load_library().sgn_elliptic_solve_fgmres(ctx.handle, net.handle, _field(ctx, h, "h"), _field(ctx, b, "b"),
                                                  _field(ctx, sigma, "sigma"), int(max_iters), ctypes.byref(info))
    _check(ctx, st, (SGN_OK, SGN_ERR_NOT_CONVERGED))
    return info


def record_sample(record, i: int):
    """(input [H][W][3], target [H][W]) views of recorder slot i."""
    H, W = record.shape[2], record.shape[3]
    flat = record[i].reshape(-1)
    return flat[:3 * H * W].view(H, W, 3), flat[3 * H * W:].view(H, W)
