"""Python binding of libfkt.so, the MI355X Fast Kernel Transform library.

Argument marshalling only: every step of the MVM runs in the library's HIP
kernels. PyTorch supplies device memory and streams. There is no CPU
fallback: if ``libfkt.so`` is missing the import of this module fails.

Entry points mirror the C ABI (include/fkt.h):
    fkt_plan(points, kernel, leaf_size, order, ...) -> Plan
    fkt_plan_batch((points, offsets), kernel, leaf_size, order, ...) -> Plan
    fkt_mvm(plan, x, y=None) -> y
    fkt_cg_solve(plan, sigma2, b, x0=None, ...) -> (x, iters, relres)
    fkt_cg_solve64(plan, sigma2, b, x0=None, ...) -> (x, iters, relres), FP64 b and x
    fkt_cg_solve_refined(plan64, plan32, sigma2, b, x0=None, ...) -> (x, iters, outer, relres)
    fkt_cg_solve_noalloc(plan, sigma2, b, x, ...) -> (iters, relres)
    fkt_precond_coarse(plan, sigma2, landmarks)
    fkt_learn_train_cond / fkt_learn_train / fkt_learn_params / ... (learned filter)
    Graph(plan, x, y).launch(), fkt_autotune / fkt_autotune_leaf,
    fkt_radial_compression(kernel, d, order), fkt_destroy(plan)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfkt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2106_04487_amd/build.py` "
                      "(there is no fallback implementation)")

# PyTorch brings its own HIP runtime; load it first so that libfkt.so binds to
# the same runtime instance as the tensors and streams it is handed.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

KERNELS = {"gaussian": 0, "exponential": 1, "matern32": 2, "matern52": 3,
           "ratquad": 4, "cauchy": 5, "laplace": 6}
PRECISIONS = {"f64": 0, "f32": 1}
STATUS = {0: "FKT_OK", 1: "FKT_EINVAL", 2: "FKT_ENOMEM", 3: "FKT_EDEVICE", 4: "FKT_EUNSUPPORTED",
          5: "FKT_ENOTCONV"}

EXPORTED = ["fkt_default_options", "fkt_plan", "fkt_mvm", "fkt_cg_solve", "fkt_cg_solve64", "fkt_cg_solve_refined",
            "fkt_destroy",
            "fkt_last_error",
            "fkt_cg_solve_noalloc", "fkt_precond_coarse",
            "fkt_plan_info", "fkt_plan_perm", "fkt_plan_target_counts", "fkt_plan_lists", "fkt_plan_stage_times",
            "fkt_radial_compression",
            "fkt_learn_nparams", "fkt_learn_params", "fkt_learn_loss_grad", "fkt_learn_train",
            "fkt_learn_train_cond", "fkt_learn_cond_grad",
            "fkt_plan_batch", "fkt_graph_create", "fkt_graph_launch", "fkt_graph_destroy", "fkt_autotune_leaf",
            "fkt_autotune"]


class FktError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("lengthscale", ctypes.c_double), ("alpha", ctypes.c_double),
                ("variance", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("prec", ctypes.c_int), ("max_depth", ctypes.c_int),
                ("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("profile", ctypes.c_int),
                ("overlap", ctypes.c_int), ("mrhs", ctypes.c_int), ("far_mode", ctypes.c_int),
                ("compress", ctypes.c_int), ("fuse", ctypes.c_int)]


_STAT_FIELDS = ["n", "nnodes", "nleaves", "depth", "rank", "nblocks", "far_nodes", "near_entries", "far_entries",
                "near_pairs", "near_lane_pairs", "far_pairs", "far_lane_pairs", "s2m_terms"]


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in _STAT_FIELDS] + [("plan_seconds", ctypes.c_double),
                                                               ("cg_fallback_iter", ctypes.c_int64),
                                                               ("radial_rank", ctypes.c_int64)]


_P = ctypes.c_void_p
_lib.fkt_default_options.argtypes = [ctypes.POINTER(_Options)]
_lib.fkt_plan.restype = ctypes.c_int
_lib.fkt_plan.argtypes = [_P, ctypes.c_int64, ctypes.c_int, _Kernel, ctypes.c_int, ctypes.c_int,
                          ctypes.POINTER(_Options), ctypes.POINTER(_P)]
_lib.fkt_mvm.restype = ctypes.c_int
_lib.fkt_mvm.argtypes = [_P, _P, _P, ctypes.c_int]
_lib.fkt_cg_solve.restype = ctypes.c_int
_lib.fkt_cg_solve.argtypes = [_P, ctypes.c_double, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
_lib.fkt_precond_coarse.restype = ctypes.c_int
_lib.fkt_precond_coarse.argtypes = [_P, ctypes.c_double, _P, ctypes.c_int]
_lib.fkt_cg_solve_noalloc.restype = ctypes.c_int
_lib.fkt_cg_solve_noalloc.argtypes = _lib.fkt_cg_solve.argtypes
_lib.fkt_cg_solve64.restype = ctypes.c_int
_lib.fkt_cg_solve64.argtypes = _lib.fkt_cg_solve.argtypes
_lib.fkt_cg_solve_refined.restype = ctypes.c_int
_lib.fkt_cg_solve_refined.argtypes = [_P, _P, ctypes.c_double, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double)]
_lib.fkt_destroy.argtypes = [_P]
_lib.fkt_last_error.restype = ctypes.c_char_p
_lib.fkt_plan_info.restype = ctypes.c_int
_lib.fkt_plan_info.argtypes = [_P, ctypes.POINTER(_Stats)]
_lib.fkt_plan_perm.restype = ctypes.c_int
_lib.fkt_plan_perm.argtypes = [_P, _P]
_lib.fkt_plan_target_counts.restype = ctypes.c_int
_lib.fkt_plan_target_counts.argtypes = [_P, _P, _P, _P, _P]
_lib.fkt_radial_compression.restype = ctypes.c_int
_lib.fkt_radial_compression.argtypes = [ctypes.POINTER(_Kernel), ctypes.c_int, ctypes.c_int, _P,
                                        ctypes.POINTER(ctypes.c_int), _P]
_lib.fkt_plan_lists.restype = ctypes.c_int
_lib.fkt_plan_lists.argtypes = [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
_lib.fkt_plan_stage_times.restype = ctypes.c_int
_lib.fkt_plan_stage_times.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
_lib.fkt_plan_batch.restype = ctypes.c_int
_lib.fkt_plan_batch.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int, _Kernel, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(_Options), ctypes.POINTER(_P)]
_lib.fkt_graph_create.restype = ctypes.c_int
_lib.fkt_graph_create.argtypes = [_P, _P, _P, ctypes.c_int, ctypes.POINTER(_P)]
_lib.fkt_graph_launch.restype = ctypes.c_int
_lib.fkt_graph_launch.argtypes = [_P]
_lib.fkt_graph_destroy.argtypes = [_P]
_lib.fkt_autotune_leaf.restype = ctypes.c_int
_lib.fkt_autotune_leaf.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _Kernel, ctypes.c_int,
                                   ctypes.POINTER(_Options), _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int), _P]
_lib.fkt_autotune.restype = ctypes.c_int
_lib.fkt_autotune.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _Kernel, ctypes.c_int,
                              ctypes.POINTER(_Options), _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _P]
_lib.fkt_learn_nparams.restype = ctypes.c_int64
_lib.fkt_learn_nparams.argtypes = []
_lib.fkt_learn_params.restype = ctypes.c_int
_lib.fkt_learn_params.argtypes = [_P, ctypes.c_double, _P, ctypes.c_int]
_lib.fkt_learn_loss_grad.restype = ctypes.c_int
_lib.fkt_learn_loss_grad.argtypes = [_P, ctypes.c_double, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _P]
_lib.fkt_learn_train_cond.restype = ctypes.c_int
_lib.fkt_learn_train_cond.argtypes = [_P, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
_lib.fkt_learn_cond_grad.restype = ctypes.c_int
_lib.fkt_learn_cond_grad.argtypes = [_P, ctypes.c_double, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _P]
_lib.fkt_learn_train.restype = ctypes.c_int
_lib.fkt_learn_train.argtypes = [_P, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int)]


def _check(status: int):
    if status != 0:
        raise FktError(status, _lib.fkt_last_error().decode())


def _stream_handle(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream or None
        return None
    if isinstance(stream, int):
        return stream or None
    return getattr(stream, "cuda_stream", None) or None


class Plan:
    """An FKT plan: tree, near/far lists and tables, resident on one device."""

    def __init__(self, handle, n, d, prec, device, stream):
        self._h = handle
        self.n, self.d, self.prec, self.device, self.stream = n, d, prec, device, stream

    @property
    def handle(self):
        if not self._h:
            raise ValueError("plan destroyed")
        return self._h

    @property
    def np_dtype(self):
        return np.float32 if self.prec == "f32" else np.float64

    def info(self) -> dict:
        s = _Stats()
        _check(_lib.fkt_plan_info(self.handle, ctypes.byref(s)))
        out = {f: int(getattr(s, f)) for f in _STAT_FIELDS}
        out["plan_seconds"] = float(s.plan_seconds)
        out["cg_fallback_iter"] = int(s.cg_fallback_iter)
        out["radial_rank"] = int(s.radial_rank)
        return out

    def perm(self) -> np.ndarray:
        p = np.zeros(self.n, dtype=np.int64)
        _check(_lib.fkt_plan_perm(self.handle, p.ctypes.data))
        return p

    def target_counts(self):
        outs = [np.zeros(self.n, dtype=np.int64) for _ in range(4)]
        _check(_lib.fkt_plan_target_counts(self.handle, *[o.ctypes.data for o in outs]))
        return tuple(outs)

    def lists(self):
        """(far_off, far_node, near_off, near_leaf): per target (caller's
        order) the far nodes and near leaves, CSR, ascending node ids."""
        nf, nq = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib.fkt_plan_lists(self.handle, None, None, None, None, ctypes.byref(nf), ctypes.byref(nq)))
        fo, no = np.zeros(self.n + 1, dtype=np.int64), np.zeros(self.n + 1, dtype=np.int64)
        fnode, nleaf = np.zeros(max(nf.value, 1), dtype=np.int64), np.zeros(max(nq.value, 1), dtype=np.int64)
        _check(_lib.fkt_plan_lists(self.handle, fo.ctypes.data, fnode.ctypes.data, no.ctypes.data, nleaf.ctypes.data,
                                   ctypes.byref(nf), ctypes.byref(nq)))
        return fo, fnode[:nf.value], no, nleaf[:nq.value]

    def stage_times(self, reset: bool = False):
        """(ms per stage summed over profiled passes, passes): stages are
        gather, s2m, m2t, near and the whole column pass ("column"). Needs a
        plan built with profile=True."""
        ms = np.zeros(5)
        calls = ctypes.c_int64(0)
        _check(_lib.fkt_plan_stage_times(self.handle, ms.ctypes.data, ctypes.byref(calls), int(reset)))
        return dict(zip(("gather", "s2m", "m2t", "near", "column"), ms.tolist())), calls.value

    def close(self):
        if self._h:
            _lib.fkt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FAR_MODES = {"auto": 0, "block": 1, "node": 2}


def _options(theta, prec, max_depth, device, stream, profile, overlap, mrhs, far_mode="auto", compress=False,
             fuse=False):
    opt = _Options()
    _lib.fkt_default_options(ctypes.byref(opt))
    opt.theta = float(theta)
    opt.prec = PRECISIONS[prec]
    opt.max_depth = int(max_depth)
    opt.device = -1 if device is None else int(device)
    opt.stream = None if device is None else _stream_handle(stream)
    opt.profile = int(bool(profile))
    opt.overlap = int(bool(overlap))
    opt.mrhs = {None: 0, "f32": 1, "bf16": 2}[mrhs]
    opt.far_mode = FAR_MODES[far_mode]
    opt.compress = int(bool(compress))
    opt.fuse = int(bool(fuse))
    return opt


def _kernel(kernel, lengthscale, alpha, variance):
    if kernel not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}; one of {sorted(KERNELS)}")
    return _Kernel(KERNELS[kernel], float(lengthscale), float(alpha), float(variance))


def _batch_points(points):
    """(concatenated FP64 rows, int64 offsets) from a list of (n_i, d) arrays
    or from an (X, offsets) pair."""
    if isinstance(points, tuple) and len(points) == 2 and np.ndim(points[1]) == 1:
        X = np.ascontiguousarray(points[0], dtype=np.float64)
        off = np.ascontiguousarray(points[1], dtype=np.int64)
    else:
        arrs = [np.asarray(p, dtype=np.float64) for p in points]
        off = np.zeros(len(arrs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([a.shape[0] for a in arrs])
        X = np.ascontiguousarray(np.concatenate(arrs, axis=0))
    return X, off


def fkt_plan_batch(points, kernel: str, leaf_size: int, order: int, *, lengthscale: float = 1.0, alpha: float = 1.0,
                   variance: float = 1.0, theta: float = 0.5, prec: str = "f64", max_depth: int = 48,
                   device: int | None = 0, stream=None, profile: bool = False, overlap: bool = True,
                   mrhs: str | None = None, far_mode: str = "auto", compress: bool = False,
                   fuse: bool = False) -> Plan:
    """One plan over independent point sets: points is a list of (n_i, d)
    arrays or (X, offsets). fkt_mvm then takes the concatenated rows."""
    X, off = _batch_points(points)
    opt = _options(theta, prec, max_depth, device, stream, profile, overlap, mrhs, far_mode, compress, fuse)
    h = _P()
    _check(_lib.fkt_plan_batch(X.ctypes.data, off.ctypes.data, len(off) - 1, X.shape[1],
                               _kernel(kernel, lengthscale, alpha, variance), int(leaf_size), int(order),
                               ctypes.byref(opt), ctypes.byref(h)))
    plan = Plan(h, X.shape[0], X.shape[1], prec, device, opt.stream)
    plan.offsets = off
    return plan


class Graph:
    """fkt_mvm(plan, x, y) captured into a HIP graph; launch() replays it on
    the plan's stream. x and y (device tensors) must stay alive."""

    def __init__(self, plan: Plan, x, y):
        self.plan, self.x, self.y = plan, x, y
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        self._h = _P()
        _check(_lib.fkt_graph_create(plan.handle, x.data_ptr(), y.data_ptr(), nrhs, ctypes.byref(self._h)))

    def launch(self):
        _check(_lib.fkt_graph_launch(self._h))

    def close(self):
        if self._h:
            _lib.fkt_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fkt_autotune_leaf(points, kernel: str, order: int, candidates, *, nrhs: int = 1, reps: int = 3,
                      lengthscale: float = 1.0, alpha: float = 1.0, variance: float = 1.0, theta: float = 0.5,
                      prec: str = "f64", batch: bool = False, device: int = 0, mrhs: str | None = None):
    """(best leaf size, {candidate: ms per MVM}) from the library's autotuner;
    points as fkt_plan, or as fkt_plan_batch with batch=True."""
    if batch:
        X, off = _batch_points(points)
        offp, ninst = off.ctypes.data, len(off) - 1
    else:
        X = np.ascontiguousarray(points, dtype=np.float64)
        off, offp, ninst = None, None, 1
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    ms = np.zeros(len(cand))
    best = ctypes.c_int(-1)
    opt = _options(theta, prec, 48, device, None, False, True, mrhs)
    _check(_lib.fkt_autotune_leaf(X.ctypes.data, offp, ninst, X.shape[0], X.shape[1],
                                  _kernel(kernel, lengthscale, alpha, variance), int(order), ctypes.byref(opt),
                                  cand.ctypes.data, len(cand), int(nrhs), int(reps), ctypes.byref(best),
                                  ms.ctypes.data))
    return best.value, dict(zip(cand.tolist(), ms.tolist()))


def fkt_autotune(points, kernel: str, order: int, leaves, far_modes=("block", "node"), *, nrhs: int = 1,
                 reps: int = 3, lengthscale: float = 1.0, alpha: float = 1.0, variance: float = 1.0,
                 theta: float = 0.5, prec: str = "f64", batch: bool = False, device: int = 0):
    """((best leaf, best far_mode name), {(leaf, far_mode): ms per MVM}) from
    the library's autotuner over leaf sizes and far-field schedules."""
    if batch:
        X, off = _batch_points(points)
        offp, ninst = off.ctypes.data, len(off) - 1
    else:
        X = np.ascontiguousarray(points, dtype=np.float64)
        off, offp, ninst = None, None, 1
    lv = np.ascontiguousarray(leaves, dtype=np.int32)
    fm = np.ascontiguousarray([FAR_MODES[m] for m in far_modes], dtype=np.int32)
    ms = np.zeros((len(lv), len(fm)))
    bl, bm = ctypes.c_int(-1), ctypes.c_int(-1)
    opt = _options(theta, prec, 48, device, None, False, True, None)
    _check(_lib.fkt_autotune(X.ctypes.data, offp, ninst, X.shape[0], X.shape[1],
                             _kernel(kernel, lengthscale, alpha, variance), int(order), ctypes.byref(opt),
                             lv.ctypes.data, len(lv), fm.ctypes.data, len(fm), int(nrhs), int(reps), ctypes.byref(bl),
                             ctypes.byref(bm), ms.ctypes.data))
    names = {v: k for k, v in FAR_MODES.items()}
    table = {(int(l), m): float(ms[i, j]) for i, l in enumerate(lv) for j, m in enumerate(far_modes)}
    return (bl.value, names[bm.value]), table


def fkt_plan(points, kernel: str, leaf_size: int, order: int, *, lengthscale: float = 1.0, alpha: float = 1.0,
             variance: float = 1.0, theta: float = 0.5, prec: str = "f64", max_depth: int = 48,
             device: int | None = 0, stream=None, profile: bool = False, overlap: bool = True,
             mrhs: str | None = None, far_mode: str = "auto", compress: bool = False,
             fuse: bool = False) -> Plan:
    """Build a plan. points: (n, d) array-like (host or device; copied to host
    FP64 for the tree build). device=None builds a host-only plan. overlap
    runs the near field on a second stream beside the far field. mrhs ("f32"
    or "bf16", FP32 plans) runs the near field of groups of 32 right-hand
    sides on the matrix cores. far_mode: "block" (target-block jobs, moments
    in LDS), "node" (one far node per wave, scalar moments, atomics) or
    "auto". compress: radial compression (exponential, Laplace, Gaussian;
    info()["radial_rank"] gives the terms per node evaluated). fuse: near
    and far field in one persistent launch."""
    if hasattr(points, "detach"):
        points = points.detach().to("cpu").double().numpy()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    if pts.ndim != 2:
        raise ValueError("points must be (n, d)")
    n, d = pts.shape
    if kernel not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}; one of {sorted(KERNELS)}")
    if prec not in PRECISIONS:
        raise ValueError(f"prec must be one of {sorted(PRECISIONS)}")
    k = _Kernel(KERNELS[kernel], float(lengthscale), float(alpha), float(variance))
    opt = _Options()
    _lib.fkt_default_options(ctypes.byref(opt))
    opt.theta = float(theta)
    opt.prec = PRECISIONS[prec]
    opt.max_depth = int(max_depth)
    opt.device = -1 if device is None else int(device)
    sh = None if device is None else _stream_handle(stream)
    opt.stream = sh
    opt.profile = int(bool(profile))
    opt.overlap = int(bool(overlap))
    opt.mrhs = {None: 0, "f32": 1, "bf16": 2}[mrhs]
    opt.far_mode = FAR_MODES[far_mode]
    opt.compress = int(bool(compress))
    opt.fuse = int(bool(fuse))
    h = _P()
    _check(_lib.fkt_plan(pts.ctypes.data, n, d, k, int(leaf_size), int(order), ctypes.byref(opt), ctypes.byref(h)))
    return Plan(h, n, d, prec, device, sh)


def _device_matrix(plan: Plan, t, name, f64=False):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    want = torch.float32 if plan.prec == "f32" and not f64 else torch.float64
    if t.dtype != want:
        raise TypeError(f"{name} must be {want} for a {plan.prec} plan")
    if t.shape[0] != plan.n or t.dim() not in (1, 2):
        raise ValueError(f"{name} must be (n,) or (n, nrhs) with n = {plan.n}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def fkt_mvm(plan: Plan, x, y=None):
    """y = K~ x on the plan's stream (asynchronous). x: (n,) or (n, nrhs)."""
    import torch
    x = _device_matrix(plan, x, "x")
    if y is None:
        y = torch.empty_like(x)
    y = _device_matrix(plan, y, "y")
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    _check(_lib.fkt_mvm(plan.handle, x.data_ptr(), y.data_ptr(), nrhs))
    return y


PRECONDS = {"none": 0, "block_jacobi": 1, "learned": 2}


def fkt_cg_solve(plan: Plan, sigma2: float, b, x0=None, *, rtol: float = 1e-6, maxit: int = 1000,
                 precond=0, _f64=False):
    """Solve (K~ + sigma2 I) x = b by CG. precond: 0/"none", 1/"block_jacobi",
    2/"learned". Returns (x, iters, relres); if maxit is reached raises
    FktError(FKT_ENOTCONV) carrying .x, .iters, .relres."""
    precond = PRECONDS[precond] if isinstance(precond, str) else int(precond)
    import torch
    b = _device_matrix(plan, b, "b", _f64)
    x = torch.zeros_like(b) if x0 is None else _device_matrix(plan, x0, "x0", _f64).clone()
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    fn = _lib.fkt_cg_solve64 if _f64 else _lib.fkt_cg_solve
    st = fn(plan.handle, float(sigma2), b.data_ptr(), x.data_ptr(), nrhs, float(rtol), int(maxit), int(precond),
            ctypes.byref(it), ctypes.byref(rr))
    if st == 5:  # FKT_ENOTCONV: x holds the last iterate
        err = FktError(st, _lib.fkt_last_error().decode())
        err.x, err.iters, err.relres = x, it.value, rr.value
        raise err
    _check(st)
    return x, it.value, rr.value


def fkt_precond_coarse(plan: Plan, sigma2: float, landmarks):
    """Two-level preconditioning at sigma2 from the given landmark indices
    (caller's order; an empty list returns to one-level)."""
    lm = np.ascontiguousarray(np.asarray(landmarks, dtype=np.int64).ravel())
    _check(_lib.fkt_precond_coarse(plan.handle, float(sigma2), lm.ctypes.data if lm.size else None, int(lm.size)))


def fkt_cg_solve_noalloc(plan: Plan, sigma2: float, b, x, *, rtol: float = 1e-6, maxit: int = 1000, precond=0):
    """fkt_cg_solve without any device allocation, in the library or here:
    x (a device tensor of b's shape and dtype, the initial guess) is
    overwritten with the solution. Returns (iters, relres); raises FktError
    (FKT_ENOTCONV carries .iters and .relres)."""
    precond = PRECONDS[precond] if isinstance(precond, str) else int(precond)
    b = _device_matrix(plan, b, "b")
    x = _device_matrix(plan, x, "x")
    if b.shape != x.shape:
        raise ValueError("b and x must have the same shape")
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = _lib.fkt_cg_solve_noalloc(plan.handle, float(sigma2), b.data_ptr(), x.data_ptr(), nrhs, float(rtol),
                                   int(maxit), int(precond), ctypes.byref(it), ctypes.byref(rr))
    if st == 5:
        err = FktError(st, _lib.fkt_last_error().decode())
        err.iters, err.relres = it.value, rr.value
        raise err
    _check(st)
    return it.value, rr.value


def fkt_cg_solve64(plan: Plan, sigma2: float, b, x0=None, *, rtol: float = 1e-6, maxit: int = 1000,
                   precond=0):
    """fkt_cg_solve with FP64 b and x for any plan: on an FP32 plan the MVMs
    run in FP32 and the solution is returned in FP64 (mixed precision)."""
    return fkt_cg_solve(plan, sigma2, b, x0, rtol=rtol, maxit=maxit, precond=precond, _f64=True)


def fkt_cg_solve_refined(plan: Plan, lo: Plan, sigma2: float, b, x0=None, *, rtol: float = 1e-6,
                         maxit: int = 1000, precond=0):
    """Mixed-precision CG: FP32 MVMs on lo (an FP32 plan over the same
    points), residual replaced by plan's FP64 one after every tenfold drop.
    b, x: FP64. Returns (x, iters, outer = replacements, relres) with relres
    the FP64 relative residual; raises FktError(FKT_ENOTCONV) carrying .x,
    .iters, .outer, .relres."""
    precond = PRECONDS[precond] if isinstance(precond, str) else int(precond)
    import torch
    b = _device_matrix(plan, b, "b")
    x = torch.zeros_like(b) if x0 is None else _device_matrix(plan, x0, "x0").clone()
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    it, ot, rr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    st = _lib.fkt_cg_solve_refined(plan.handle, lo.handle, float(sigma2), b.data_ptr(), x.data_ptr(), nrhs,
                                   float(rtol), int(maxit), int(precond), ctypes.byref(it), ctypes.byref(ot),
                                   ctypes.byref(rr))
    if st == 5:
        err = FktError(st, _lib.fkt_last_error().decode())
        err.x, err.iters, err.outer, err.relres = x, it.value, ot.value, rr.value
        raise err
    _check(st)
    return x, it.value, ot.value, rr.value


def fkt_learn_nparams() -> int:
    return int(_lib.fkt_learn_nparams())


def fkt_learn_params(plan: Plan, sigma2: float, params=None) -> np.ndarray:
    """Current weights of the learned preconditioner (FP32 vector); with
    params given, replaces them first."""
    buf = np.zeros(fkt_learn_nparams(), dtype=np.float32)
    if params is not None:
        buf[:] = np.asarray(params, dtype=np.float32)
        _check(_lib.fkt_learn_params(plan.handle, float(sigma2), buf.ctypes.data, 1))
    _check(_lib.fkt_learn_params(plan.handle, float(sigma2), buf.ctypes.data, 0))
    return buf


def fkt_learn_loss_grad(plan: Plan, sigma2: float, v):
    """(loss, gradient) of the learned preconditioner's training objective
    for the batch v (n x B, FP64; host or device)."""
    import torch
    v = torch.as_tensor(v, dtype=torch.float64, device="cuda")
    if v.dim() == 1:
        v = v[:, None]
    v = v.contiguous()
    loss = ctypes.c_double(0.0)
    grad = np.zeros(fkt_learn_nparams(), dtype=np.float32)
    _check(_lib.fkt_learn_loss_grad(plan.handle, float(sigma2), v.data_ptr(), v.shape[1], ctypes.byref(loss),
                                    grad.ctypes.data))
    return loss.value, grad


def fkt_learn_train(plan: Plan, sigma2: float, steps: int, batch: int = 8, lr: float = 1e-3, seed: int = 1,
                    judge_iters: int = 0):
    """Adam steps on device-drawn Gaussian batches; with judge_iters > 0
    block-Jacobi judges the result (see fkt.h). Returns (loss of the first
    step, loss of the last step, accepted)."""
    l0 = ctypes.c_double(float("nan"))
    l1 = ctypes.c_double(float("nan"))
    acc = ctypes.c_int(1)
    _check(_lib.fkt_learn_train(plan.handle, float(sigma2), int(steps), int(batch), float(lr), int(seed),
                                ctypes.byref(l0), ctypes.byref(l1), int(judge_iters), ctypes.byref(acc)))
    return l0.value, l1.value, bool(acc.value)


def fkt_learn_train_cond(plan: Plan, sigma2: float, steps: int, lanczos: int = 30, lr: float = 1e-2, seed: int = 1,
                         judge_iters: int = 0):
    """Adam steps on the condition number of the preconditioned operator
    (Lanczos from PCG); returns (kappa_first, kappa_last, accepted)."""
    c0, c1, acc = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_int(1)
    _check(_lib.fkt_learn_train_cond(plan.handle, float(sigma2), int(steps), int(lanczos), float(lr), int(seed),
                                     ctypes.byref(c0), ctypes.byref(c1), int(judge_iters), ctypes.byref(acc)))
    return c0.value, c1.value, bool(acc.value)


def fkt_learn_cond_grad(plan: Plan, sigma2: float, b, lanczos: int = 30):
    """(kappa estimate, gradient of log kappa) for the right-hand side b."""
    import torch
    b = torch.as_tensor(b, dtype=torch.float64, device="cuda").contiguous()
    c = ctypes.c_double(0.0)
    g = np.zeros(fkt_learn_nparams(), dtype=np.float32)
    _check(_lib.fkt_learn_cond_grad(plan.handle, float(sigma2), b.data_ptr(), int(lanczos), ctypes.byref(c),
                                    g.ctypes.data))
    return c.value, g


def fkt_radial_compression(kernel: str, d: int, order: int, *, lengthscale: float = 1.0, alpha: float = 1.0,
                           variance: float = 1.0):
    """(ranks R_k, rows kept per degree by the compressed kernels (0: none),
    interpolative coefficients [k][jj][i] or None) for the kernel."""
    k = _kernel(kernel, lengthscale, alpha, variance)
    mj = order // 2 + 1
    rk = np.zeros(order + 1, dtype=np.int32)
    keep = ctypes.c_int(0)
    coef = np.zeros((order + 1, mj, mj), dtype=np.float64)
    _check(_lib.fkt_radial_compression(ctypes.byref(k), int(d), int(order), rk.ctypes.data, ctypes.byref(keep),
                                       coef.ctypes.data))
    return rk.tolist(), keep.value, (coef if keep.value > 0 else None)


def fkt_destroy(plan: Plan):
    plan.close()


def last_error() -> str:
    return _lib.fkt_last_error().decode()
