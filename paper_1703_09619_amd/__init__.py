"""Product-to-sum element-matrix fill on AMD Instinct MI355X (gfx950).

Thin ctypes binding of the C ABI in include/p2s.h (argument marshalling
only; every stage of the fill runs in the HIP kernels of libp2s.so).
PyTorch supplies device memory and the stream.

    import torch, paper_1703_09619_amd as p2s
    ctx = p2s.Context(0)
    plan = ctx.plan(p2s.VECTOR, p2s.MAT_ROTDIAG, orders, quad)
    out, status = plan.execute(nodes_dev, material_dev)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2s.so")

SCALAR, VECTOR = 0, 1
MAT_SINCOSEXP, MAT_ROTDIAG, MAT_PLANEWAVE, ALPHA_SAMPLED = 0, 1, 2, 3
FP64, SPLIT_FP32, SPLIT_INT8 = 0, 1, 2
METHOD_P2S, METHOD_DIRECT, METHOD_DIRECT_SF = 0, 1, 2
OUTPUT_DENSE, OUTPUT_PACKED_UPPER = 0, 1
FAM_PHI, FAM_DPHI, FAM_PSI = 0, 1, 2
STATUS_DETJ, STATUS_NONFINITE, STATUS_FALLBACK = 1, 2, 4
MAX_ORDER, MAX_Q = 8, 32

# every symbol the C ABI exports (include/p2s.h)
EXPORTS = (
    "p2s_create", "p2s_destroy", "p2s_last_error", "p2s_num_dofs", "p2s_layout", "p2s_layout_output",
    "p2s_plan_create", "p2s_plan_execute", "p2s_plan_workspace_bytes", "p2s_plan_destroy",
    "p2s_fill_element_matrices", "p2s_plan_coupling", "p2s_plan_moments",
    "p2s_gauss_rule", "p2s_linearization", "p2s_plan_profile", "p2s_plan_profile_read",
    "p2s_plan_set_schedule", "p2s_plan_get_schedule", "p2s_plan_autotune", "p2s_plan_capture",
    "p2s_plan_replay", "p2s_mlp_init", "p2s_mlp_set_params", "p2s_mlp_get_params", "p2s_mlp_save",
    "p2s_mlp_load", "p2s_features", "p2s_mlp_forward", "p2s_mlp_gradients", "p2s_mlp_train_step",
    "p2s_mlp_predict", "p2s_plan_set_learned", "p2s_plan_rules", "p2s_rel_error", "p2s_plan_tail_values",
    "p2s_plan_tail_records", "p2s_fill_uniform_noalloc", "p2s_cheb2d_num_dofs", "p2s_cheb2d_create",
    "p2s_cheb2d_execute", "p2s_cheb2d_profile", "p2s_cheb2d_destroy", "p2s_context_device",
)
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 85, 128, 57, 34873
KMIN, KMAX = 6, 24


class P2SError(RuntimeError):
    pass


class _Terms(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("material", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("method", ctypes.c_int32),
                ("stiff_scale", ctypes.c_double), ("mass_scale", ctypes.c_double),
                ("output", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def load():
    """Load libp2s.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise P2SError("libp2s.so is not built: run `python -m paper_1703_09619_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        lib.p2s_create.argtypes = [ctypes.POINTER(vp), i32]
        lib.p2s_destroy.argtypes = [vp]
        lib.p2s_destroy.restype = None
        lib.p2s_last_error.argtypes = [vp]
        lib.p2s_last_error.restype = ctypes.c_char_p
        lib.p2s_num_dofs.argtypes = [i32, i32]
        lib.p2s_num_dofs.restype = i64
        lib.p2s_layout.argtypes = [i32, i64, vp, vp]
        lib.p2s_layout_output.argtypes = [i32, i32, i64, vp, vp]
        lib.p2s_plan_create.argtypes = [vp, ctypes.POINTER(_Terms), i64, vp, vp, ctypes.POINTER(vp)]
        lib.p2s_plan_execute.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.p2s_plan_workspace_bytes.argtypes = [vp]
        lib.p2s_plan_workspace_bytes.restype = i64
        lib.p2s_plan_destroy.argtypes = [vp]
        lib.p2s_plan_destroy.restype = None
        lib.p2s_fill_element_matrices.argtypes = [vp, ctypes.POINTER(_Terms), i64, vp, vp, vp, vp, vp, vp, vp]
        lib.p2s_fill_uniform_noalloc.argtypes = [vp, ctypes.POINTER(_Terms), i64, i32, i32, i32, i32, vp, vp, vp,
                                                 vp, vp]
        lib.p2s_cheb2d_num_dofs.argtypes = [i32]
        lib.p2s_cheb2d_num_dofs.restype = i64
        lib.p2s_cheb2d_create.argtypes = [vp, i64, i32, i32, ctypes.POINTER(vp)]
        lib.p2s_cheb2d_execute.argtypes = [vp, i32, vp, vp, d, d, vp, vp, vp]
        lib.p2s_cheb2d_profile.argtypes = [vp, i32, vp]
        lib.p2s_cheb2d_destroy.argtypes = [vp]
        lib.p2s_cheb2d_destroy.restype = None
        lib.p2s_context_device.argtypes = [vp]
        lib.p2s_plan_coupling.argtypes = [vp, vp, vp, vp, vp]
        lib.p2s_plan_moments.argtypes = [vp, vp, vp, vp, vp]
        lib.p2s_plan_profile.argtypes = [vp, i32]
        lib.p2s_plan_profile_read.argtypes = [vp, vp, vp]
        lib.p2s_plan_set_schedule.argtypes = [vp, i32, i32]
        lib.p2s_plan_get_schedule.argtypes = [vp, vp, vp]
        lib.p2s_plan_autotune.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_char_p, vp]
        lib.p2s_plan_capture.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.p2s_plan_replay.argtypes = [vp, vp]
        lib.p2s_mlp_init.argtypes = [vp, ctypes.c_uint64, i64]
        lib.p2s_mlp_set_params.argtypes = [vp, vp]
        lib.p2s_mlp_get_params.argtypes = [vp, vp]
        lib.p2s_mlp_save.argtypes = [vp, ctypes.c_char_p]
        lib.p2s_mlp_load.argtypes = [vp, ctypes.c_char_p]
        lib.p2s_features.argtypes = [vp, i32, i64, vp, vp, vp, vp]
        lib.p2s_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
        lib.p2s_mlp_gradients.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        lib.p2s_mlp_train_step.argtypes = [vp, i64, vp, vp, ctypes.c_float, vp, vp]
        lib.p2s_mlp_predict.argtypes = [vp, i64, vp, ctypes.c_float, vp, vp]
        lib.p2s_plan_set_learned.argtypes = [vp, i32, ctypes.c_float, i32, d]
        lib.p2s_plan_rules.argtypes = [vp, vp]
        lib.p2s_plan_tail_values.argtypes = [vp, vp]
        lib.p2s_plan_tail_records.argtypes = [vp, vp, vp, vp, vp]
        lib.p2s_rel_error.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp]
        lib.p2s_gauss_rule.argtypes = [i32, vp, vp]
        lib.p2s_linearization.argtypes = [i32, i32, i32, i32, vp]
        for f in ("p2s_create", "p2s_layout", "p2s_layout_output", "p2s_plan_create", "p2s_plan_execute",
                  "p2s_fill_element_matrices", "p2s_plan_coupling", "p2s_plan_moments",
                  "p2s_gauss_rule", "p2s_linearization", "p2s_plan_profile", "p2s_plan_profile_read",
                  "p2s_plan_set_schedule", "p2s_plan_get_schedule", "p2s_plan_autotune", "p2s_plan_capture",
                  "p2s_plan_replay", "p2s_mlp_init", "p2s_mlp_set_params", "p2s_mlp_get_params",
                  "p2s_mlp_save", "p2s_mlp_load", "p2s_features", "p2s_mlp_forward", "p2s_mlp_gradients",
                  "p2s_mlp_train_step", "p2s_mlp_predict", "p2s_plan_set_learned", "p2s_plan_rules",
                  "p2s_rel_error", "p2s_plan_tail_values", "p2s_plan_tail_records",
                  "p2s_fill_uniform_noalloc", "p2s_cheb2d_create", "p2s_cheb2d_execute", "p2s_cheb2d_profile",
                  "p2s_context_device"):
            getattr(lib, f).restype = i32
        _lib = lib
    return _lib


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def num_dofs(problem: int, N: int) -> int:
    return int(load().p2s_num_dofs(problem, N))


def layout(problem: int, orders, output: int = OUTPUT_DENSE) -> np.ndarray:
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    off = np.zeros(len(orders) + 1, dtype=np.int64)
    rc = load().p2s_layout_output(problem, output, len(orders), _np_ptr(orders), _np_ptr(off))
    if rc != 0:
        raise P2SError("p2s_layout failed: %d" % rc)
    return off


def gauss_rule(Q: int):
    x = np.zeros(Q)
    w = np.zeros(Q)
    rc = load().p2s_gauss_rule(Q, _np_ptr(x), _np_ptr(w))
    if rc != 0:
        raise P2SError("p2s_gauss_rule failed: %d" % rc)
    return x, w


def linearization(xfam: int, m1: int, yfam: int, m2: int) -> np.ndarray:
    c = np.zeros(2 * MAX_ORDER)
    rc = load().p2s_linearization(xfam, m1, yfam, m2, _np_ptr(c))
    if rc != 0:
        raise P2SError("p2s_linearization failed: %d" % rc)
    return c


def terms(problem: int, material: int, precision: int = FP64, method: int = METHOD_P2S,
          stiff_scale: float = 1.0, mass_scale: float = 1.0, output: int = OUTPUT_DENSE) -> _Terms:
    return _Terms(problem, material, precision, method, stiff_scale, mass_scale, output, 0)


class Context:
    """A library context on one GPU (tables built once)."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.p2s_create(ctypes.byref(h), device)
        if rc != 0:
            raise P2SError("p2s_create failed (%d): %s" % (rc, lib.p2s_last_error(None).decode()))
        self._h = h
        self.device = device

    def error(self) -> str:
        return load().p2s_last_error(self._h).decode()

    def check(self, rc: int, what: str):
        if rc != 0:
            raise P2SError("%s failed (%d): %s" % (what, rc, self.error()))

    def close(self):
        if getattr(self, "_h", None):
            load().p2s_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- learned quadrature order (network held by the context)
    def mlp_init(self, seed: int = 0, max_batch: int = 4096):
        self.check(load().p2s_mlp_init(self._h, seed, max_batch), "p2s_mlp_init")

    def mlp_params(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, np.float32)
        self.check(load().p2s_mlp_get_params(self._h, _np_ptr(p)), "p2s_mlp_get_params")
        return p

    def mlp_set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == MLP_PARAMS
        self.check(load().p2s_mlp_set_params(self._h, _np_ptr(p)), "p2s_mlp_set_params")

    def mlp_save(self, path: str):
        self.check(load().p2s_mlp_save(self._h, path.encode()), "p2s_mlp_save")

    def mlp_load(self, path: str):
        self.check(load().p2s_mlp_load(self._h, path.encode()), "p2s_mlp_load")

    def features(self, material, nodes, mat, stream=None):
        import torch
        E = nodes.shape[0]
        x = torch.empty((E, MLP_IN), dtype=torch.float32, device=nodes.device)
        self.check(load().p2s_features(self._h, material, E, _dev_ptr(nodes), _dev_ptr(mat), _dev_ptr(x),
                                       _stream(stream)), "p2s_features")
        return x

    def mlp_forward(self, x, stream=None):
        import torch
        z = torch.empty((x.shape[0], MLP_OUT), dtype=torch.float32, device=x.device)
        self.check(load().p2s_mlp_forward(self._h, x.shape[0], _dev_ptr(x), _dev_ptr(z), _stream(stream)),
                   "p2s_mlp_forward")
        return z

    def mlp_gradients(self, x, labels, stream=None):
        """(loss sum, gradient of the mean loss) for a batch."""
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self.check(load().p2s_mlp_gradients(self._h, x.shape[0], _dev_ptr(x), _dev_ptr(labels), _dev_ptr(g),
                                            _dev_ptr(loss), _stream(stream)), "p2s_mlp_gradients")
        return loss, g

    def mlp_train_step(self, x, labels, lr, loss, stream=None):
        self.check(load().p2s_mlp_train_step(self._h, x.shape[0], _dev_ptr(x), _dev_ptr(labels), float(lr),
                                             _dev_ptr(loss), _stream(stream)), "p2s_mlp_train_step")

    def mlp_predict(self, x, p_cover=0.99, stream=None):
        import torch
        q = torch.empty((x.shape[0], 3), dtype=torch.int32, device=x.device)
        self.check(load().p2s_mlp_predict(self._h, x.shape[0], _dev_ptr(x), float(p_cover), _dev_ptr(q),
                                          _stream(stream)), "p2s_mlp_predict")
        return q

    def rel_error(self, a, b, offsets=None, block=0, stream=None):
        """Per-element ||a-b||/||b|| of device blocks (offsets: device int64 [E+1])."""
        import torch
        E = (offsets.numel() - 1) if offsets is not None else a.numel() // block
        err = torch.empty(E, dtype=torch.float64, device=a.device)
        self.check(load().p2s_rel_error(self._h, E, block, _dev_ptr(offsets), _dev_ptr(a), _dev_ptr(b),
                                        _dev_ptr(err), _stream(stream)), "p2s_rel_error")
        return err

    def fill_element_matrices(self, problem, material_kind, nodes, material, orders, quad, out=None,
                              status=None, precision=FP64, method=METHOD_P2S, stiff_scale=1.0, mass_scale=1.0,
                              stream=None):
        """p2s_fill_element_matrices: the one-shot fill (plans cached per
        batch shape in the context).  Returns (out, status)."""
        import torch
        t = terms(problem, material_kind, precision, method, stiff_scale, mass_scale)
        orders = np.ascontiguousarray(orders, dtype=np.int32)
        quad = np.ascontiguousarray(quad, dtype=np.int32).reshape(-1, 3)
        E = len(orders)
        dev = torch.device("cuda", self.device)
        if out is None:
            out = torch.empty(int(layout(problem, orders)[-1]) if E else 0, dtype=torch.float64, device=dev)
        if status is None:
            status = torch.empty(E, dtype=torch.int32, device=dev)
        rc = load().p2s_fill_element_matrices(self._h, ctypes.byref(t), E, _dev_ptr(nodes), _dev_ptr(material),
                                              _np_ptr(orders), _np_ptr(quad), _dev_ptr(out), _dev_ptr(status),
                                              _stream(stream))
        self.check(rc, "p2s_fill_element_matrices")
        return out, status

    def fill_uniform_noalloc(self, problem, material_kind, nodes, material, E, N, Q, out, status,
                             stiff_scale=1.0, mass_scale=1.0, stream=None):
        """p2s_fill_uniform_noalloc: E elements of order N and rule Q (3
        points per axis) through the library's fixed device scratch; out and
        status are caller-allocated device tensors."""
        t = terms(problem, material_kind, FP64, METHOD_P2S, stiff_scale, mass_scale)
        Qu, Qv, Qw = (int(q) for q in Q)
        rc = load().p2s_fill_uniform_noalloc(self._h, ctypes.byref(t), int(E), int(N), Qu, Qv, Qw,
                                             _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(out),
                                             _dev_ptr(status), _stream(stream))
        self.check(rc, "p2s_fill_uniform_noalloc")

    def cheb2d(self, E, M, Q) -> "Cheb2D":
        return Cheb2D(self, E, M, Q)

    def plan(self, problem, material, orders, quad, precision=FP64, method=METHOD_P2S,
             stiff_scale=1.0, mass_scale=1.0, output=OUTPUT_DENSE) -> "Plan":
        return Plan(self, terms(problem, material, precision, method, stiff_scale, mass_scale, output), orders,
                    quad)


class Plan:
    """Schedule + workspace for one batch shape; execute() allocates nothing
    in the library (the output tensors are allocated by torch unless given)."""

    def __init__(self, ctx: Context, t: _Terms, orders, quad):
        self.ctx = ctx
        self.terms = t
        self.orders = np.ascontiguousarray(orders, dtype=np.int32)
        self.quad = np.ascontiguousarray(quad, dtype=np.int32).reshape(-1, 3)
        self.E = len(self.orders)
        h = ctypes.c_void_p()
        rc = load().p2s_plan_create(ctx._h, ctypes.byref(t), self.E, _np_ptr(self.orders),
                                    _np_ptr(self.quad), ctypes.byref(h))
        ctx.check(rc, "p2s_plan_create")
        self._h = h
        self.offsets = layout(t.problem, self.orders, t.output) if self.E else np.zeros(1, np.int64)

    @property
    def workspace_bytes(self) -> int:
        return int(load().p2s_plan_workspace_bytes(self._h))

    def execute(self, nodes, material, out=None, status=None, stream=None):
        import torch
        dev = torch.device("cuda", self.ctx.device)
        if out is None:
            out = torch.empty(int(self.offsets[-1]), dtype=torch.float64, device=dev)
        if status is None:
            status = torch.empty(self.E, dtype=torch.int32, device=dev)
        rc = load().p2s_plan_execute(self._h, _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(out),
                                     _dev_ptr(status), _stream(stream))
        self.ctx.check(rc, "p2s_plan_execute")
        return out, status

    def profile(self, enable: bool = True):
        """Record HIP events around each stage launch of later executions."""
        self.ctx.check(load().p2s_plan_profile(self._h, int(enable)), "p2s_plan_profile")

    def profile_read(self):
        """{stage: (ms, launches)} since the last read, stages coupling,
        moments, contraction, other."""
        ms = np.zeros(4)
        n = np.zeros(4, dtype=np.int64)
        self.ctx.check(load().p2s_plan_profile_read(self._h, _np_ptr(ms), _np_ptr(n)), "p2s_plan_profile_read")
        names = ("coupling", "moments", "contraction", "other")
        return {names[i]: (float(ms[i]), int(n[i])) for i in range(4)}

    def set_schedule(self, mode: int, wgs_per_cu: int = 1):
        self.ctx.check(load().p2s_plan_set_schedule(self._h, mode, wgs_per_cu), "p2s_plan_set_schedule")

    def schedule(self):
        m = np.zeros(1, np.int32)
        w = np.zeros(1, np.int32)
        self.ctx.check(load().p2s_plan_get_schedule(self._h, _np_ptr(m), _np_ptr(w)), "p2s_plan_get_schedule")
        return int(m[0]), int(w[0])

    def autotune(self, nodes, material, out, status, cache_path=None, stream=None):
        """Pick the fastest schedule on these buffers; returns its ms."""
        best = np.zeros(1)
        cp = cache_path.encode() if cache_path else None
        rc = load().p2s_plan_autotune(self._h, _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(out),
                                      _dev_ptr(status), _stream(stream), cp, _np_ptr(best))
        self.ctx.check(rc, "p2s_plan_autotune")
        return float(best[0])

    def capture(self, nodes, material, out, status, stream):
        """Record one execution into a HIP graph (stream: a torch.cuda.Stream)."""
        rc = load().p2s_plan_capture(self._h, _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(out),
                                     _dev_ptr(status), ctypes.c_void_p(stream.cuda_stream))
        self.ctx.check(rc, "p2s_plan_capture")

    def replay(self, stream=None):
        self.ctx.check(load().p2s_plan_replay(self._h, _stream(stream)), "p2s_plan_replay")

    def set_learned(self, enable=True, p_cover=0.99, theta=1e-9, k_direct=KMAX + 1):
        self.ctx.check(load().p2s_plan_set_learned(self._h, int(enable), float(p_cover), int(k_direct),
                                                   float(theta)), "p2s_plan_set_learned")

    def tail_values(self) -> np.ndarray:
        t = np.zeros(self.E)
        self.ctx.check(load().p2s_plan_tail_values(self._h, _np_ptr(t)), "p2s_plan_tail_values")
        return t

    def rules(self) -> np.ndarray:
        q = np.zeros((self.E, 3), np.int32)
        self.ctx.check(load().p2s_plan_rules(self._h, _np_ptr(q)), "p2s_plan_rules")
        return q

    def coupling(self, nodes, material, stream=None):
        import torch
        F = 7 if self.terms.problem == SCALAR else 12
        P = int(np.prod(self.quad[0])) if self.E else 0
        a = torch.empty(self.E * F * P, dtype=torch.float64, device=torch.device("cuda", self.ctx.device))
        rc = load().p2s_plan_coupling(self._h, _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(a), _stream(stream))
        self.ctx.check(rc, "p2s_plan_coupling")
        return a.view(self.E, F, P)

    def moments(self, nodes, material, stream=None):
        import torch
        F = 7 if self.terms.problem == SCALAR else 12
        K = 2 * int(self.orders[0]) - 1 if self.E else 1
        m = torch.empty(self.E * F * K ** 3, dtype=torch.float64, device=torch.device("cuda", self.ctx.device))
        rc = load().p2s_plan_moments(self._h, _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(m), _stream(stream))
        self.ctx.check(rc, "p2s_plan_moments")
        return m.view(self.E, F, K, K, K)

    def tail_records(self, nodes, material, stream=None):
        """[E][F][16] tail records of the moment stage at the plan's rules."""
        import torch
        F = 7 if self.terms.problem == SCALAR else 12
        r = torch.zeros(self.E * F * 16, dtype=torch.float64, device=torch.device("cuda", self.ctx.device))
        rc = load().p2s_plan_tail_records(self._h, _dev_ptr(nodes), _dev_ptr(material), _dev_ptr(r), _stream(stream))
        self.ctx.check(rc, "p2s_plan_tail_records")
        return r.view(self.E, F, 16)

    def close(self):
        if getattr(self, "_h", None):
            load().p2s_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cheb2D:
    """The paper's 2-D Chebyshev example (p2s_cheb2d_*): workspace for E
    elements of order M = N with Q x Q Gauss points."""

    def __init__(self, ctx: Context, E: int, M: int, Q: int):
        self.ctx, self.E, self.M, self.Q = ctx, int(E), int(M), int(Q)
        h = ctypes.c_void_p()
        rc = load().p2s_cheb2d_create(ctx._h, self.E, self.M, self.Q, ctypes.byref(h))
        if rc != 0:
            raise P2SError("p2s_cheb2d_create failed (%d)" % rc)
        self._h = h
        self.ndof = int(load().p2s_cheb2d_num_dofs(self.M))

    def execute(self, nodes, material, method=METHOD_P2S, stiff_scale=1.0, mass_scale=1.0, out=None,
                status=None, stream=None):
        import torch
        dev = torch.device("cuda", self.ctx.device)
        if out is None:
            out = torch.empty(self.E * self.ndof * self.ndof, dtype=torch.float64, device=dev)
        if status is None:
            status = torch.empty(self.E, dtype=torch.int32, device=dev)
        rc = load().p2s_cheb2d_execute(self._h, int(method), _dev_ptr(nodes), _dev_ptr(material),
                                       float(stiff_scale), float(mass_scale), _dev_ptr(out), _dev_ptr(status),
                                       _stream(stream))
        if rc != 0:
            raise P2SError("p2s_cheb2d_execute failed (%d)" % rc)
        return out, status

    def profile(self, enable=True):
        """Mean ms per execution of (geometry, moments, contraction or
        direct) since the last call; then enable or disable timing."""
        ms = np.zeros(3)
        load().p2s_cheb2d_profile(self._h, int(enable), _np_ptr(ms))
        return ms

    def close(self):
        if getattr(self, "_h", None):
            load().p2s_cheb2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fill(ctx: Context, problem, material_kind, nodes, material, orders, quad, **kw):
    """One-shot fill with device tensors; returns (out, offsets, status)."""
    p = ctx.plan(problem, material_kind, orders, quad, **kw)
    out, status = p.execute(nodes, material)
    return out, p.offsets, status
