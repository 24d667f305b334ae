"""Plain FP64 CPU oracle for the hierarchical element-matrix fill.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark import this package.  The product library never
imports it, and it shares no code with the product library (it is a separate C
file compiled with gcc, plus this ctypes wrapper).

The oracle fills every entry of the element matrix by direct, full 3-D tensor
Gauss-Legendre quadrature of eq. (2) of the paper (Section II), i.e. the
direct numerical integration the paper compares against (Section IV).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCALAR, VECTOR = 0, 1
MAT_SINCOSEXP, MAT_ROTDIAG, MAT_PLANEWAVE, ALPHA_SAMPLED = 0, 1, 2, 3
STATUS_DETJ, STATUS_NONFINITE = 1, 2

_lib = None
_native = None

# IEEE FP64 without value-changing optimizations: no fast-math, no FMA
# contraction (the oracle's sums round exactly as written)
_FP_FLAGS = ["-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (portable -O2 build, the
    one the tests load; it travels with the tree to other hosts)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2"] + _FP_FLAGS + ["-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def build_native(directory: str) -> str:
    """Compile oracle.c with -O3 -march=native for the host it runs on, into
    `directory` (the timed CPU baseline; the same source and FP64 rules as
    the test build, vectorized for this CPU)."""
    path = os.path.join(directory, "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native"] + _FP_FLAGS + ["-o", path, _SRC, "-lm"])
    return path


def use_native(directory: str) -> None:
    """Make fill() run the -O3 -march=native build from build_native()."""
    global _native
    _native = _bind(ctypes.CDLL(build_native(directory)))


def _load(native: bool = False):
    global _lib
    if native:
        if _native is None:
            raise RuntimeError("use_native() has not been called")
        return _native
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    d, i, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_gauss_legendre.argtypes = [i, vp, vp]
    lib.oracle_gauss_legendre.restype = i
    for f in ("oracle_phi", "oracle_dphi", "oracle_psi"):
        getattr(lib, f).argtypes = [i, d]
        getattr(lib, f).restype = d
    lib.oracle_map.argtypes = [vp, d, d, d, vp, vp]
    lib.oracle_map.restype = None
    lib.oracle_eps.argtypes = [i, vp, vp, vp]
    lib.oracle_eps.restype = None
    lib.oracle_coupling.argtypes = [i, i, vp, vp, i, i, i, vp]
    lib.oracle_coupling.restype = d
    lib.oracle_fill.argtypes = [i, i, i64, vp, vp, vp, vp, vp, d, d, vp, vp, i]
    lib.oracle_fill.restype = i
    lib.oracle_moments.argtypes = [i, i, vp, vp, i, i, i, i, vp]
    lib.oracle_moments.restype = i
    lib.oracle_num_dofs.argtypes = [i, i]
    lib.oracle_num_dofs.restype = i64
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def gauss_legendre(Q: int):
    lib = _load()
    x = np.zeros(Q)
    w = np.zeros(Q)
    if lib.oracle_gauss_legendre(Q, _ptr(x), _ptr(w)) != 0:
        raise ValueError("bad Q")
    return x, w


def phi(m: int, t: float) -> float:
    return _load().oracle_phi(m, t)


def dphi(m: int, t: float) -> float:
    return _load().oracle_dphi(m, t)


def psi(m: int, t: float) -> float:
    return _load().oracle_psi(m, t)


def geometry(nodes: np.ndarray, u: float, v: float, w: float):
    """x and J[r][c] = dx_r/du_c of the triquadratic map of one element."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    x = np.zeros(3)
    J = np.zeros((3, 3))
    _load().oracle_map(_ptr(nodes), u, v, w, _ptr(x), _ptr(J))
    return x, J


def permittivity(material: int, params, x):
    """3x3 permittivity tensor of an analytic material at physical point x."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    eps = np.zeros((3, 3))
    _load().oracle_eps(material, _ptr(params), _ptr(x), _ptr(eps))
    return eps


def num_dofs(problem: int, N: int) -> int:
    return N ** 3 if problem == SCALAR else 3 * (N - 1) * N * N


def num_fields(problem: int) -> int:
    return 7 if problem == SCALAR else 12


def coupling(problem, material, params, nodes, Qu, Qv, Qw):
    """Coupling fields at the Gauss points of one element, [F][Qu*Qv*Qw]."""
    F = num_fields(problem)
    out = np.zeros((F, Qu * Qv * Qw))
    params = np.ascontiguousarray(params, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    _load().oracle_coupling(problem, material, _ptr(params), _ptr(nodes), Qu, Qv, Qw, _ptr(out))
    return out


def moments(problem, material, params, nodes, Qu, Qv, Qw, K):
    """Plain-definition moment tensors of eq. (4), [F][K][K][K]."""
    F = num_fields(problem)
    out = np.zeros((F, K, K, K))
    params = np.ascontiguousarray(params, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    rc = _load().oracle_moments(problem, material, _ptr(params), _ptr(nodes), Qu, Qv, Qw, K, _ptr(out))
    if rc != 0:
        raise ValueError("oracle_moments failed: %d" % rc)
    return out


def layout(problem: int, orders) -> np.ndarray:
    orders = np.asarray(orders)
    sizes = np.array([num_dofs(problem, int(n)) ** 2 for n in orders], dtype=np.int64)
    off = np.zeros(len(orders) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def fill(problem, material, nodes, mat, orders, quad, s_K=1.0, s_M=1.0, nthreads=0, native=False):
    """Element matrices by direct quadrature (nthreads OpenMP threads over
    elements, 0 = OpenMP's default; native: the build_native() library).

    Returns (out, offsets, status): out is the concatenation of the dense
    row-major FP64 blocks, offsets[E+1] their starts.
    """
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    mat = np.ascontiguousarray(mat, dtype=np.float64)
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    quad = np.ascontiguousarray(quad, dtype=np.int32)
    E = orders.shape[0]
    off = layout(problem, orders)
    out = np.zeros(int(off[-1]))
    status = np.zeros(E, dtype=np.uint32)
    rc = _load(native).oracle_fill(problem, material, E, _ptr(nodes), _ptr(mat), _ptr(orders),
                             _ptr(quad), _ptr(off), float(s_K), float(s_M),
                             _ptr(out), _ptr(status), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_fill rejected its arguments: %d" % rc)
    return out, off, status


def blocks(out: np.ndarray, off: np.ndarray, e: int) -> np.ndarray:
    """Element e's matrix as a square 2-D array."""
    n = int(round((off[e + 1] - off[e]) ** 0.5))
    return out[off[e]:off[e + 1]].reshape(n, n)
