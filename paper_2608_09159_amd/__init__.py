"""Python binding of libpdhcg.so, the MI355X (gfx950) restarted-PDHG solver for
conic convex QP.

The binding only marshals arguments: every step of the solve runs in the HIP
library.  There is no CPU fallback; importing works without the library, but
any call raises ``RuntimeError`` when ``libpdhcg.so`` is missing.

Functions mirror the C ABI of ``include/pdhcg.h``:

    default_settings(**overrides) -> Settings
    setup(problem, settings) -> Handle       (pdhcg_setup, count == 1)
    Handle.solve(x0=None, y0=None) -> dict    (pdhcg_solve)
    setup_batch(problems, settings) -> BatchHandle   (pdhcg_setup, count > 1)
    BatchHandle.solve(x0s=None, y0s=None) -> [dict]  (pdhcg_solve_batch)
    Handle.trace(count) -> dict               (pdhcg_get_trace)
    Handle.scaling() -> dict                  (pdhcg_get_scaling)
    Handle.free()                             (pdhcg_free)
    project_cones(kind, r, metric, alpha)     (pdhcg_project_cones, diagnostic)
    project_cones_noalloc(kind, r, out, ...)  (pdhcg_project_cones_noalloc: device
                                               tensors, no allocation)
    MLP(dims, max_batch).forward / .train_step / .set_params / .get_params /
        .grads / .free                        (pdhcg_mlp_*: the warm-start
                                               network's BF16 matrix-core kernels)

``problem`` is any object with the fields of ``instances.Problem``
(n, m, A as scipy CSR, b, c, optional P / R / D, cones as
(type, start, dim, alpha) tuples with type in CONE_CODES, optional row
bounds row_lo / row_hi and box bounds x_lo / x_hi).

``memory_kind="device"`` passes every problem array, warm start and output
to the library as device memory (torch CUDA tensors; numpy inputs are moved
to the device first) and returns x, y, s as torch CUDA tensors;
``allocator="torch"`` makes the library take its device memory from torch's
caching allocator (settings.dev_alloc / dev_free).

``interleave`` takes a name of ORDER (or the PDHCG_ORDER_* value): the
device's coordinate order; "auto" (the default) picks "degree" for large
cone-free problems with skewed columns.  Inputs and outputs stay in the
caller's order either way.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdhcg.so")

CONE_CODES = {"free": 0, "nonneg": 1, "soc": 2, "rsoc": 3, "exp": 4, "pow": 5, "box": 6, "exp1": 7}
STATUS = {1: "OPTIMAL", 2: "MAX_ITER", 3: "TIME_LIMIT", 4: "NUMERICAL", 5: "ABORTED"}
SCHEMES = {"rh": 0, "avg": 1}
INNER = {"jacobi": 0, "euclid": 1}
PRECISION = {"fp64": 0, "fp32": 1}
CONE_SCALING = {"block": 0, "rescaled": 1}
MEMORY_KIND = {"host": 0, "device": 1}
ORDER = {"caller": -1, "auto": 0, "cones": 1, "degree": 2}   # settings.interleave

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class ProblemC(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32),
                ("A_rowptr", _i64p), ("A_col", _i32p), ("A_val", _dp),
                ("b", _dp), ("c", _dp),
                ("P_rowptr", _i64p), ("P_col", _i32p), ("P_val", _dp),
                ("r", C.c_int32), ("R", _dp), ("D", _dp),
                ("nblocks", C.c_int32), ("cone_type", _i32p), ("cone_start", _i32p),
                ("cone_dim", _i32p), ("cone_alpha", _dp),
                ("row_lo", _dp), ("row_hi", _dp), ("x_lo", _dp), ("x_hi", _dp)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None                      # NULL: the library reports PDHCG_E_MEM


def _torch_free(ptr, stream, ctx):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


# module-level, so the callbacks outlive every handle that uses them
TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
TORCH_FREE = _FREE_FN(_torch_free)


class Settings(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("time_limit", C.c_double),
                ("check_every", C.c_int32), ("scheme", C.c_int32), ("rho", C.c_double),
                ("avg_epoch", C.c_int32), ("inner", C.c_int32), ("fixed_inner", C.c_int32),
                ("j_max", C.c_int32), ("eps_in0", C.c_double), ("gamma_in", C.c_double),
                ("eps_min", C.c_double), ("beta_s", C.c_double), ("beta_n", C.c_double),
                ("beta_a", C.c_double), ("pid_beta_i", C.c_double), ("pid_kp", C.c_double),
                ("pid_ki", C.c_double), ("pid_kd", C.c_double), ("scaling", C.c_int32),
                ("ruiz_iters", C.c_int32), ("pock_chambolle", C.c_int32),
                ("pc_alpha", C.c_double), ("bound_objective", C.c_int32),
                ("power_iters", C.c_int32), ("a_norm", C.c_double), ("omega0", C.c_double),
                ("precision", C.c_int32), ("trace_iters", C.c_int32), ("block_dim", C.c_int32),
                ("grid_dim", C.c_int32), ("lanes_at", C.c_int32), ("lanes_a", C.c_int32),
                ("host_poll", C.c_int32), ("stream", C.c_void_p), ("verbose", C.c_int32),
                ("time_kernels", C.c_int32), ("autotune", C.c_int32),
                ("tune_iters", C.c_int32), ("fp32_tol", C.c_double),
                ("interleave", C.c_int32), ("cone_scaling", C.c_int32),
                ("memory_kind", C.c_int32), ("dev_alloc", _ALLOC_FN), ("dev_free", _FREE_FN),
                ("alloc_ctx", C.c_void_p)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int64),
                ("inner_iterations", C.c_int64), ("restarts", C.c_int64),
                ("rel_primal", C.c_double), ("rel_dual", C.c_double), ("rel_gap", C.c_double),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("setup_s", C.c_double), ("solve_s", C.c_double), ("omega", C.c_double),
                ("a_norm", C.c_double), ("x", _dp), ("y", _dp), ("s", _dp),
                ("kernel_s", C.c_double), ("kernel_launches", C.c_int64),
                ("grid_dim", C.c_int32), ("block_dim", C.c_int32),
                ("polish_iterations", C.c_int64)]


class TraceC(C.Structure):
    _fields_ = [("count", C.c_int32), ("x", _dp), ("y", _dp), ("wx", _dp), ("wy", _dp),
                ("tau", _dp), ("sigma", _dp), ("omega", _dp), ("eps_in", _dp),
                ("inner", _i32p), ("restart", _i32p), ("check", _i32p), ("E", _dp)]


_LIB = None

EXPORTS = ("pdhcg_default_settings", "pdhcg_setup", "pdhcg_solve", "pdhcg_solve_batch",
           "pdhcg_get_trace", "pdhcg_get_scaling", "pdhcg_free", "pdhcg_strerror",
           "pdhcg_version", "pdhcg_last_cone_failure", "pdhcg_project_cones",
           "pdhcg_project_cones_noalloc", "pdhcg_mlp_create", "pdhcg_mlp_set_params", "pdhcg_mlp_get_params",
           "pdhcg_mlp_forward", "pdhcg_mlp_train_step", "pdhcg_mlp_get_grads", "pdhcg_mlp_free")


class AdamC(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


def lib_path():
    return LIB_PATH


def load(path=None):
    """Load libpdhcg.so (raises RuntimeError if it has not been built)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libpdhcg.so not found at {p}; build it with "
                           "`python -m paper_2608_09159_amd.build` (hipcc, gfx950)")
    # torch bundles its own HIP runtime under the same soname as the one this
    # library links; loading torch first makes the process use one runtime
    # (loaded the other way round, torch later finds no GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(p)
    lib.pdhcg_default_settings.argtypes = [C.POINTER(Settings)]
    lib.pdhcg_setup.argtypes = [C.POINTER(ProblemC), C.c_int32, C.POINTER(Settings),
                                C.POINTER(C.c_void_p)]
    lib.pdhcg_solve.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(ResultC)]
    lib.pdhcg_solve_batch.argtypes = [C.c_void_p, C.POINTER(_dp), C.POINTER(_dp),
                                      C.POINTER(ResultC)]
    lib.pdhcg_get_trace.argtypes = [C.c_void_p, C.c_int32, C.POINTER(TraceC)]
    lib.pdhcg_get_scaling.argtypes = [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.pdhcg_free.argtypes = [C.c_void_p]
    lib.pdhcg_free.restype = None
    lib.pdhcg_strerror.argtypes = [C.c_int]
    lib.pdhcg_strerror.restype = C.c_char_p
    lib.pdhcg_version.restype = C.c_char_p
    lib.pdhcg_last_cone_failure.argtypes = [_dp, C.POINTER(C.c_int64)]
    lib.pdhcg_project_cones.argtypes = [C.c_int32, C.c_int32, C.c_int64, _dp, _dp, _dp, _dp]
    lib.pdhcg_project_cones_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_void_p,
                                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    _fp = C.POINTER(C.c_float)
    lib.pdhcg_mlp_create.argtypes = [C.c_int32, _i32p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.pdhcg_mlp_set_params.argtypes = [C.c_void_p, C.c_int32, _fp, _fp]
    lib.pdhcg_mlp_get_params.argtypes = [C.c_void_p, C.c_int32, _fp, _fp]
    lib.pdhcg_mlp_get_grads.argtypes = [C.c_void_p, C.c_int32, _fp, _fp]
    lib.pdhcg_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.pdhcg_mlp_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                         C.POINTER(AdamC), C.POINTER(C.c_double)]
    lib.pdhcg_mlp_free.argtypes = [C.c_void_p]
    lib.pdhcg_mlp_free.restype = None
    if path is None:
        _LIB = lib
    return lib


def _check(rc, what):
    if rc != 0:
        msg = load().pdhcg_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} ({rc})")


def default_settings(**kw) -> Settings:
    s = Settings()
    _check(load().pdhcg_default_settings(C.byref(s)), "pdhcg_default_settings")
    for k, v in kw.items():
        if k == "scheme":
            v = SCHEMES[v] if isinstance(v, str) else v
        elif k == "inner":
            v = INNER[v] if isinstance(v, str) else v
        elif k == "precision":
            v = PRECISION[v] if isinstance(v, str) else v
        elif k == "cone_scaling":
            v = CONE_SCALING[v] if isinstance(v, str) else v
        elif k == "memory_kind":
            v = MEMORY_KIND[v] if isinstance(v, str) else v
        elif k == "interleave":
            v = ORDER[v] if isinstance(v, str) else v
        elif k == "allocator":
            if v == "torch":
                s.dev_alloc, s.dev_free = TORCH_ALLOC, TORCH_FREE
            elif v is not None:
                raise ValueError(f"allocator {v!r}: 'torch' or None")
            continue
        elif k == "stream":
            v = getattr(v, "cuda_stream", v)
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


def _ptr(a, ctype):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):           # a torch tensor: its device address
        return C.cast(C.c_void_p(a.data_ptr()), C.POINTER(ctype))
    return a.ctypes.data_as(C.POINTER(ctype))


_TORCH_DT = {np.float64: "float64", np.int64: "int64", np.int32: "int32"}


def _on_device(x, dt):
    """x (numpy array, sequence or torch tensor) as a contiguous torch CUDA
    tensor of dtype dt."""
    import torch
    tdt = getattr(torch, _TORCH_DT[dt])
    if hasattr(x, "data_ptr"):
        return x.to(device="cuda", dtype=tdt).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _is_device(settings):
    return settings is not None and settings.memory_kind == MEMORY_KIND["device"]


class _Marshalled:
    """Keeps the argument buffers alive for the duration of pdhcg_setup
    (numpy arrays, or torch CUDA tensors with device memory)."""

    def __init__(self, prob, device=False):
        A = prob.A.tocsr()
        self.keep = []

        def arr(x, dt):
            if x is None:
                return None
            y = _on_device(x, dt) if device else np.ascontiguousarray(x, dtype=dt)
            self.keep.append(y)
            return y

        pc = ProblemC()
        pc.n, pc.m = int(prob.n), int(prob.m)
        pc.A_rowptr = _ptr(arr(A.indptr, np.int64), C.c_int64)
        pc.A_col = _ptr(arr(A.indices, np.int32), C.c_int32)
        pc.A_val = _ptr(arr(A.data, np.float64), C.c_double)
        pc.b = _ptr(arr(prob.b, np.float64), C.c_double)
        pc.c = _ptr(arr(prob.c, np.float64), C.c_double)
        if prob.P is not None:
            P = prob.P.tocsr()
            pc.P_rowptr = _ptr(arr(P.indptr, np.int64), C.c_int64)
            pc.P_col = _ptr(arr(P.indices, np.int32), C.c_int32)
            pc.P_val = _ptr(arr(P.data, np.float64), C.c_double)
        if prob.R is not None:
            pc.r = int(prob.R.shape[0])
            pc.R = _ptr(arr(prob.R, np.float64), C.c_double)
            pc.D = _ptr(arr(prob.D, np.float64), C.c_double) if prob.D is not None else None
        ct = np.array([CONE_CODES[k] for k, _, _, _ in prob.cones], dtype=np.int32)
        pc.nblocks = len(prob.cones)
        pc.cone_type = _ptr(arr(ct, np.int32), C.c_int32)
        pc.cone_start = _ptr(arr([s for _, s, _, _ in prob.cones], np.int32), C.c_int32)
        pc.cone_dim = _ptr(arr([d for _, _, d, _ in prob.cones], np.int32), C.c_int32)
        pc.cone_alpha = _ptr(arr([a for _, _, _, a in prob.cones], np.float64), C.c_double)
        if getattr(prob, "row_lo", None) is not None:
            pc.row_lo = _ptr(arr(prob.row_lo, np.float64), C.c_double)
            pc.row_hi = _ptr(arr(prob.row_hi, np.float64), C.c_double)
        if getattr(prob, "x_lo", None) is not None:
            pc.x_lo = _ptr(arr(prob.x_lo, np.float64), C.c_double)
            pc.x_hi = _ptr(arr(prob.x_hi, np.float64), C.c_double)
        self.pc = pc


class Handle:
    def __init__(self, ptr, prob, settings):
        self.ptr = ptr
        self.n, self.m = int(prob.n), int(prob.m)
        self.settings = settings

    def solve(self, x0=None, y0=None, want_s=False):
        lib = load()
        res = ResultC()
        dev = _is_device(self.settings)
        vec = _vec_factory(dev)
        x = vec(self.n)
        y = vec(self.m)
        s = vec(self.n) if want_s else None
        res.x = _ptr(x, C.c_double)
        res.y = _ptr(y, C.c_double)
        res.s = _ptr(s, C.c_double) if want_s else None
        x0a = _as_input(x0, dev)
        y0a = _as_input(y0, dev)
        _check(lib.pdhcg_solve(self.ptr, _ptr(x0a, C.c_double), _ptr(y0a, C.c_double),
                               C.byref(res)), "pdhcg_solve")
        return _result_dict(res, x, y, s)

    def trace(self, count, inst=0):
        lib = load()
        n, m = self._dims(inst)
        t = TraceC()
        t.count = count
        bufs = dict(x=np.zeros((count, n)), y=np.zeros((count, m)),
                    wx=np.zeros((count, n)), wy=np.zeros((count, m)),
                    tau=np.zeros(count), sigma=np.zeros(count), omega=np.zeros(count),
                    eps_in=np.zeros(count), E=np.zeros(count))
        ibufs = dict(inner=np.zeros(count, np.int32), restart=np.zeros(count, np.int32),
                     check=np.zeros(count, np.int32))
        for k, v in bufs.items():
            setattr(t, k, _ptr(v, C.c_double))
        for k, v in ibufs.items():
            setattr(t, k, _ptr(v, C.c_int32))
        _check(lib.pdhcg_get_trace(self.ptr, inst, C.byref(t)), "pdhcg_get_trace")
        out = {k: v[:t.count] for k, v in {**bufs, **ibufs}.items()}
        out["count"] = t.count
        return out

    def _dims(self, inst):
        if inst != 0:
            raise IndexError(inst)
        return self.n, self.m

    def scaling(self, inst=0):
        lib = load()
        n, m = self._dims(inst)
        Sx, Sy = np.zeros(n), np.zeros(m)
        vals = [C.c_double() for _ in range(4)]
        _check(lib.pdhcg_get_scaling(self.ptr, inst, _ptr(Sx, C.c_double), _ptr(Sy, C.c_double),
                                     *[C.pointer(v) for v in vals]), "pdhcg_get_scaling")
        return dict(Sx=Sx, Sy=Sy, nu_b=vals[0].value, nu_c=vals[1].value, eta=vals[2].value,
                    omega0=vals[3].value)

    def free(self):
        if self.ptr:
            load().pdhcg_free(self.ptr)
            self.ptr = None

    def __del__(self):
        # at interpreter exit a Python allocator (torch's) may already be
        # gone: leave the memory to the process end then
        if sys.is_finalizing() and self.settings is not None and self.settings.dev_free:
            return
        try:
            self.free()
        except Exception:
            pass


def _vec_factory(device):
    if not device:
        return lambda k: np.zeros(k)
    import torch
    return lambda k: torch.zeros(max(k, 0), dtype=torch.float64, device="cuda")


def _as_input(v, device):
    if v is None:
        return None
    return _on_device(v, np.float64) if device else np.ascontiguousarray(v, dtype=np.float64)


def _result_dict(res, x, y, s):
    out = dict(status=STATUS.get(res.status, str(res.status)), iterations=res.iterations,
               inner_iterations=res.inner_iterations, restarts=res.restarts,
               rel_primal=res.rel_primal, rel_dual=res.rel_dual, rel_gap=res.rel_gap,
               primal_obj=res.primal_obj, dual_obj=res.dual_obj, setup_s=res.setup_s,
               solve_s=res.solve_s, omega=res.omega, a_norm=res.a_norm, x=x, y=y,
               kernel_s=res.kernel_s, kernel_launches=res.kernel_launches,
               grid_dim=res.grid_dim, block_dim=res.block_dim,
               polish_iterations=res.polish_iterations)
    if s is not None:
        out["s"] = s
    return out


def last_cone_failure():
    """(count, record) of failed cone root-finding in the last solve:
    record = (cone type, r0, r1, r2, m0, m1, m2, alpha)."""
    rec = np.zeros(8)
    cnt = C.c_int64()
    _check(load().pdhcg_last_cone_failure(_ptr(rec, C.c_double), C.byref(cnt)),
           "pdhcg_last_cone_failure")
    return int(cnt.value), rec


def project_cones(kind, r, metric=None, alpha=None):
    """pdhcg_project_cones: r is a (count, dim) array of blocks of one cone
    type (name or code); metric the same shape or None; alpha (count,) for
    POW.  Returns the projected blocks."""
    code = CONE_CODES[kind] if isinstance(kind, str) else int(kind)
    r = np.ascontiguousarray(r, dtype=np.float64)
    if r.ndim != 2:
        raise ValueError("r must be (count, dim)")
    count, dim = r.shape
    m = None if metric is None else np.ascontiguousarray(metric, dtype=np.float64)
    if m is not None and m.shape != r.shape:
        raise ValueError("metric must have the shape of r")
    a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
    if a is not None and a.shape != (count,):
        raise ValueError("alpha must have one entry per block")
    out = np.empty_like(r)
    _check(load().pdhcg_project_cones(code, dim, count, _ptr(a, C.c_double), _ptr(r, C.c_double),
                                      _ptr(m, C.c_double), _ptr(out, C.c_double)),
           "pdhcg_project_cones")
    return out


def project_cones_noalloc(kind, r, out, metric=None, alpha=None, stream=None):
    """pdhcg_project_cones_noalloc on torch CUDA float64 tensors: r and out
    (count, dim), metric the same shape or None, alpha (count,) for POW;
    issued on `stream` (a torch stream, or None for the null stream) without
    any allocation.  Returns out."""
    code = CONE_CODES[kind] if isinstance(kind, str) else int(kind)

    def dev(t, shape):
        if t is None:
            return None
        if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8
                and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected a contiguous CUDA float64 tensor of shape {shape}")
        return t.data_ptr()

    count, dim = int(r.shape[0]), int(r.shape[1])
    st = getattr(stream, "cuda_stream", stream)
    _check(load().pdhcg_project_cones_noalloc(code, dim, count, dev(alpha, (count,)), dev(r, (count, dim)),
                                              dev(metric, (count, dim)), dev(out, (count, dim)), st),
           "pdhcg_project_cones_noalloc")
    return out


class BatchHandle(Handle):
    """Handle of a batch (pdhcg_setup with count > 1)."""

    def __init__(self, ptr, probs, settings):
        self.ptr = ptr
        self.ns = [int(p.n) for p in probs]
        self.ms = [int(p.m) for p in probs]
        self.count = len(probs)
        self.settings = settings

    def _dims(self, inst):
        return self.ns[inst], self.ms[inst]

    def solve(self, x0s=None, y0s=None, want_s=False):
        """pdhcg_solve_batch: one persistent launch for every instance.
        x0s / y0s: None or sequences of per-instance arrays (or None)."""
        lib = load()
        res = (ResultC * self.count)()
        dev = _is_device(self.settings)
        vec = _vec_factory(dev)
        xs = [vec(n) for n in self.ns]
        ys = [vec(m) for m in self.ms]
        ss = [vec(n) for n in self.ns] if want_s else [None] * self.count
        for i in range(self.count):
            res[i].x = _ptr(xs[i], C.c_double)
            res[i].y = _ptr(ys[i], C.c_double)
            res[i].s = _ptr(ss[i], C.c_double) if want_s else None
        keep = []

        def ptr_array(vs):
            if vs is None:
                return None
            arr = (_dp * self.count)()
            for i, v in enumerate(vs):
                if v is not None:
                    a = _as_input(v, dev)
                    keep.append(a)
                    arr[i] = _ptr(a, C.c_double)
            return arr

        _check(lib.pdhcg_solve_batch(self.ptr, ptr_array(x0s), ptr_array(y0s), res),
               "pdhcg_solve_batch")
        return [_result_dict(res[i], xs[i], ys[i], ss[i]) for i in range(self.count)]


def setup_batch(probs, settings=None, **kw) -> BatchHandle:
    """pdhcg_setup with count = len(probs) > 1."""
    lib = load()
    probs = list(probs)
    if len(probs) < 2:
        raise ValueError("a batch needs at least two problems; use setup() for one")
    s = settings if settings is not None else default_settings(**kw)
    ms = [_Marshalled(p, _is_device(s)) for p in probs]
    arr = (ProblemC * len(probs))(*[m.pc for m in ms])
    h = C.c_void_p()
    _check(lib.pdhcg_setup(arr, len(probs), C.byref(s), C.byref(h)), "pdhcg_setup")
    return BatchHandle(h.value, probs, s)


def setup(prob, settings=None, **kw) -> Handle:
    lib = load()
    s = settings if settings is not None else default_settings(**kw)
    m = _Marshalled(prob, _is_device(s))
    h = C.c_void_p()
    _check(lib.pdhcg_setup(C.byref(m.pc), 1, C.byref(s), C.byref(h)), "pdhcg_setup")
    return Handle(h.value, prob, s)


def solve(prob, x0=None, y0=None, want_s=False, **kw):
    """Convenience: setup + solve + free."""
    h = setup(prob, **kw)
    try:
        return h.solve(x0, y0, want_s=want_s)
    finally:
        h.free()


class MLP:
    """The warm-start network (pdhcg_mlp_*): ReLU MLP with BF16 matrix
    operands, FP32 master weights and Adam.  Inputs and targets are torch
    CUDA float32 tensors (device pointers); parameters are numpy arrays."""

    def __init__(self, dims, max_batch, stream=None):
        lib = load()
        self.dims = [int(d) for d in dims]
        self.layers = len(self.dims) - 1
        self.max_batch = int(max_batch)
        arr = np.ascontiguousarray(self.dims, dtype=np.int32)
        h = C.c_void_p()
        st = getattr(stream, "cuda_stream", stream)
        _check(lib.pdhcg_mlp_create(self.layers, _ptr(arr, C.c_int32), self.max_batch, st,
                                    C.byref(h)), "pdhcg_mlp_create")
        self.ptr = h.value

    def set_params(self, layer, W, b):
        W = np.ascontiguousarray(W, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        assert W.shape == (self.dims[layer], self.dims[layer + 1]) and b.shape == (self.dims[layer + 1],)
        _check(load().pdhcg_mlp_set_params(self.ptr, layer, _ptr(W, C.c_float), _ptr(b, C.c_float)),
               "pdhcg_mlp_set_params")

    def get_params(self, layer):
        W = np.zeros((self.dims[layer], self.dims[layer + 1]), dtype=np.float32)
        b = np.zeros(self.dims[layer + 1], dtype=np.float32)
        _check(load().pdhcg_mlp_get_params(self.ptr, layer, _ptr(W, C.c_float), _ptr(b, C.c_float)),
               "pdhcg_mlp_get_params")
        return W, b

    def grads(self, layer):
        dW = np.zeros((self.dims[layer], self.dims[layer + 1]), dtype=np.float32)
        db = np.zeros(self.dims[layer + 1], dtype=np.float32)
        _check(load().pdhcg_mlp_get_grads(self.ptr, layer, _ptr(dW, C.c_float), _ptr(db, C.c_float)),
               "pdhcg_mlp_get_grads")
        return dW, db

    @staticmethod
    def _dev(t, cols):
        if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4
                and t.is_contiguous() and t.dim() == 2 and t.shape[1] == cols):
            raise ValueError("expected a contiguous CUDA float32 tensor with %d columns" % cols)
        return t.data_ptr()

    def forward(self, x, out=None):
        import torch
        B = int(x.shape[0])
        if out is None:
            out = torch.empty((B, self.dims[-1]), dtype=torch.float32, device=x.device)
        _check(load().pdhcg_mlp_forward(self.ptr, self._dev(x, self.dims[0]), B,
                                        self._dev(out, self.dims[-1])), "pdhcg_mlp_forward")
        return out

    def train_step(self, x, y, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, update=True):
        """One step on (x, y); returns the batch loss before the update."""
        B = int(x.shape[0])
        opt = AdamC(lr, beta1, beta2, eps) if update else None
        loss = C.c_double()
        _check(load().pdhcg_mlp_train_step(self.ptr, self._dev(x, self.dims[0]),
                                           self._dev(y, self.dims[-1]), B,
                                           C.byref(opt) if opt is not None else None,
                                           C.byref(loss)), "pdhcg_mlp_train_step")
        return loss.value

    def free(self):
        if self.ptr:
            load().pdhcg_mlp_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
