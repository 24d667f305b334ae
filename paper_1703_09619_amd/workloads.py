"""Seeded synthetic workloads for the element-matrix fill.

This module only draws inputs: element nodes, material parameters, orders and
quadrature sizes.  It holds none of the fill's arithmetic (no basis, no
coupling factors, no moments, no contraction), so the CPU oracle and the GPU
path can both consume its output without sharing any computation.

The one geometric computation here is an input-acceptance rule: a perturbed
triquadratic element is accepted only if the Jacobian determinant of its map
stays above a tenth of the nominal value on a check grid.  Otherwise its node
noise is shrunk by 0.8 and re-checked.  Plain i.i.d. node noise at the stated
amplitudes inverts many elements (a tangled element has no meaningful
matrix), so some such rule is needed; it only decides which inputs are used.

Workload recipes (the paper's own experiment is a 2-D mesh whose figures are
not available; these stand in for 3-D curved inhomogeneous hexahedra):

  scalar_sincos   scalar diffusion+mass, eps = 1 + 0.5 sin(k x) cos(k y) e^-z
  vector_rotdiag  curl-curl+mass, eps = R^T diag(1 + 0.5 sin(k.x + 2 pi a/3)) R
  scalar_mixed    scalar, N ~ U{2..8}, Q = 2N, k ~ U[pi, 4 pi]
  scalar_planewave scalar, eps = 1 + 0.8 sin(k.x + phase), |k| log-uniform
"""
from __future__ import annotations

import numpy as np

SCALAR, VECTOR = 0, 1
MAT_SINCOSEXP, MAT_ROTDIAG, MAT_PLANEWAVE, ALPHA_SAMPLED = 0, 1, 2, 3

BASE_SEED = 1703096190
NOMINAL_DETJ = 0.125  # the unperturbed map x = (u+1)/2 has J = I/2


def nominal_nodes() -> np.ndarray:
    """[27][3] node positions of the unit cube, node (i,j,k) at i+3j+9k."""
    n = np.zeros((27, 3))
    for k in range(3):
        for j in range(3):
            for i in range(3):
                n[i + 3 * j + 9 * k] = (0.5 * i, 0.5 * j, 0.5 * k)
    return n


def _lagrange_d(t):
    """Quadratic Lagrange values and derivatives on {-1,0,1} at points t."""
    t = np.asarray(t, dtype=np.float64)
    l = np.stack([0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)], -1)
    d = np.stack([t - 0.5, -2.0 * t, t + 0.5], -1)
    return l, d


def _check_points(extra_q=()):
    g = np.linspace(-1.0, 1.0, 9)
    pts = [np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)]
    for q in extra_q:
        x = np.polynomial.legendre.leggauss(int(q))[0]
        pts.append(np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3))
    return np.concatenate(pts, 0)


def _min_detj(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Minimum Jacobian determinant of each element over the check points
    (input acceptance only)."""
    lu, du = _lagrange_d(pts[:, 0])
    lv, dv = _lagrange_d(pts[:, 1])
    lw, dw = _lagrange_d(pts[:, 2])
    # shape derivative weights [P][27][3]
    gu = np.einsum("pi,pj,pk->pkji", du, lv, lw).reshape(len(pts), 27)
    gv = np.einsum("pi,pj,pk->pkji", lu, dv, lw).reshape(len(pts), 27)
    gw = np.einsum("pi,pj,pk->pkji", lu, lv, dw).reshape(len(pts), 27)
    G = np.stack([gu, gv, gw], 1).reshape(3 * len(pts), 27)  # row p*3+c
    out = np.empty(nodes.shape[0])
    for s in range(0, nodes.shape[0], 512):
        X = nodes[s:s + 512]  # [e][27][r]
        J = np.matmul(G[None], X).reshape(X.shape[0], len(pts), 3, 3)  # [e][p][c][r]
        d = (J[..., 0, 0] * (J[..., 1, 1] * J[..., 2, 2] - J[..., 1, 2] * J[..., 2, 1])
             - J[..., 0, 1] * (J[..., 1, 0] * J[..., 2, 2] - J[..., 1, 2] * J[..., 2, 0])
             + J[..., 0, 2] * (J[..., 1, 0] * J[..., 2, 1] - J[..., 1, 1] * J[..., 2, 0]))
        out[s:s + 512] = d.min(axis=1)
    return out


def perturbed_nodes(rng: np.random.Generator, E: int, amplitude, check_q=(),
                    min_ratio: float = 0.1, shrink: float = 0.8):
    """Nominal unit-cube nodes plus i.i.d. U[-a, a] noise on every coordinate.

    `amplitude` is a scalar or an [E] array.  Elements failing the acceptance
    rule have their noise scaled by `shrink` until they pass.  Returns
    (nodes [E][27][3], effective amplitude [E], number of shrink steps [E]).
    """
    amp = np.broadcast_to(np.asarray(amplitude, dtype=np.float64), (E,)).copy()
    noise = rng.uniform(-1.0, 1.0, size=(E, 27, 3)) * amp[:, None, None]
    base = nominal_nodes()[None]
    pts = _check_points(check_q)
    steps = np.zeros(E, dtype=np.int32)
    todo = np.arange(E)
    while todo.size:
        md = _min_detj(base + noise[todo], pts)
        bad = md <= min_ratio * NOMINAL_DETJ
        todo = todo[bad]
        noise[todo] *= shrink
        amp[todo] *= shrink
        steps[todo] += 1
    return base + noise, amp, steps


def haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation: QR of a Gaussian matrix, sign-fixed."""
    A = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


class Workload(dict):
    """Inputs of one fill call (a dict with attribute access)."""
    __getattr__ = dict.__getitem__


def make(name: str, E: int | None = None, seed: int | None = None, N: int | None = None,
         Q: int | None = None) -> Workload:
    """Build one of the named workloads.

    names: 'scalar_n4' (64 elements, N=4, Q=8), 'vector_n6' (4096, N=6, Q=12),
    'scalar_mixed' (20000, N~U{2..8}, Q=2N), 'vector_n8' (8192, N=8, Q=16),
    'scalar_planewave' (50000, N=6, Q=24 reference rule).
    """
    specs = {
        "scalar_n4": dict(E=64, problem=SCALAR, N=4, Q=8, amp=0.1, idx=0),
        "vector_n6": dict(E=4096, problem=VECTOR, N=6, Q=12, amp=0.15, idx=1),
        "scalar_mixed": dict(E=20000, problem=SCALAR, N=None, Q=None, amp=0.1, idx=2),
        "vector_n8": dict(E=8192, problem=VECTOR, N=8, Q=16, amp=0.15, idx=3),
        "scalar_planewave": dict(E=50000, problem=SCALAR, N=6, Q=24, amp=None, idx=4),
    }
    if name not in specs:
        raise KeyError(name)
    sp = dict(specs[name])
    if E is not None:
        sp["E"] = int(E)
    if N is not None:
        sp["N"] = int(N)
    if Q is not None:
        sp["Q"] = int(Q)
    E = sp["E"]
    rng = np.random.default_rng(BASE_SEED + sp["idx"] if seed is None else seed)
    problem = sp["problem"]

    if name == "scalar_mixed":
        orders = rng.integers(2, 9, size=E).astype(np.int32)
        quad = np.repeat((2 * orders)[:, None], 3, 1).astype(np.int32)
        nodes, amp, steps = perturbed_nodes(rng, E, sp["amp"], check_q=())
        kappa = rng.uniform(np.pi, 4 * np.pi, size=E)
        mat = kappa[:, None].copy()
        material = MAT_SINCOSEXP
    elif name == "scalar_planewave":
        orders = np.full(E, sp["N"], dtype=np.int32)
        quad = np.full((E, 3), sp["Q"], dtype=np.int32)
        a = rng.uniform(0.0, 0.3, size=E)
        nodes, amp, steps = perturbed_nodes(rng, E, a, check_q=())
        kmag = np.pi * np.exp(rng.uniform(np.log(0.5), np.log(16.0), size=E))
        kdir = unit_vectors(rng, E)
        phase = rng.uniform(0.0, 2 * np.pi, size=E)
        mat = np.concatenate([kdir * kmag[:, None], phase[:, None]], 1)
        material = MAT_PLANEWAVE
    else:
        orders = np.full(E, sp["N"], dtype=np.int32)
        quad = np.full((E, 3), sp["Q"], dtype=np.int32)
        nodes, amp, steps = perturbed_nodes(rng, E, sp["amp"], check_q=(sp["Q"],))
        if problem == SCALAR:
            mat = np.full((E, 1), 2 * np.pi)
            material = MAT_SINCOSEXP
        else:
            mat = np.zeros((E, 12))
            kmag = rng.uniform(0.0, 4 * np.pi, size=E)
            kdir = unit_vectors(rng, E)
            for e in range(E):
                mat[e, :9] = haar_rotation(rng).reshape(-1)
            mat[:, 9:12] = kdir * kmag[:, None]
            material = MAT_ROTDIAG
    return Workload(name=name, problem=problem, material=material, E=E,
                    nodes=np.ascontiguousarray(nodes), mat=np.ascontiguousarray(mat),
                    orders=orders, quad=np.ascontiguousarray(quad),
                    amp=amp, shrink_steps=steps)


def subset(w: Workload, idx) -> Workload:
    """The same workload restricted to element indices idx."""
    idx = np.asarray(idx)
    out = Workload(w)
    for k in ("nodes", "mat", "orders", "quad", "amp", "shrink_steps"):
        if k in w:
            out[k] = np.ascontiguousarray(w[k][idx])
    out["E"] = len(idx)
    return out


def num_dofs(problem: int, N: int) -> int:
    """Degrees of freedom of one element (sizes the output, not arithmetic)."""
    return N ** 3 if problem == SCALAR else 3 * (N - 1) * N * N


# ---------------------------------------------------------------------------
# The paper's 2-D example (Section III): a stand-in for the mesh of its
# Fig. 2, whose node coordinates the paper does not give.  The domain is the
# curved quadrilateral bounded by y = -f(x), y = f(x), x = -g(y), x = g(y) with
# the caption's f(x) = -0.2 (x^2 - 1)^2 + 1 and g(y) = 0.2 (y^2 - 1)^2 + 1
# (corners at (+-1, +-1)).  Transfinite (Coons) interpolation of its four
# edges maps the reference square onto it as (s, t) -> (s g(t), t f(s)),
# which is of degree 4 in each variable, so fourth-order quadrilaterals
# represent it exactly.  The square is split into nx x ny elements.

CHEB2D_MATERIAL = (2.0, 1.0, 1.0, 2.0)  # eps_r = 2 exp(x + y + 2)


def cheb2d_mesh(nx: int = 4, ny: int = 4) -> Workload:
    """nodes [nx*ny][25][2] (node (i,j) at i + 5 j on the reference points
    (-1 + i/2, -1 + j/2)) and material [nx*ny][4] of the stand-in mesh."""
    f = lambda x: -0.2 * (x * x - 1.0) ** 2 + 1.0
    g = lambda y: 0.2 * (y * y - 1.0) ** 2 + 1.0
    ref = np.array([-1.0, -0.5, 0.0, 0.5, 1.0])
    E = nx * ny
    nodes = np.zeros((E, 25, 2))
    for iy in range(ny):
        for ix in range(nx):
            e = iy * nx + ix
            s0, s1 = -1.0 + 2.0 * ix / nx, -1.0 + 2.0 * (ix + 1) / nx
            t0, t1 = -1.0 + 2.0 * iy / ny, -1.0 + 2.0 * (iy + 1) / ny
            for j in range(5):
                for i in range(5):
                    s = s0 + 0.5 * (ref[i] + 1.0) * (s1 - s0)
                    t = t0 + 0.5 * (ref[j] + 1.0) * (t1 - t0)
                    nodes[e, i + 5 * j] = (s * g(t), t * f(s))
    mat = np.tile(np.array(CHEB2D_MATERIAL), (E, 1))
    return Workload(name="cheb2d_mesh", E=E, nodes=nodes, mat=mat)


def cheb2d_replicated(copies: int) -> Workload:
    """The 16-element stand-in mesh repeated `copies` times (a larger batch
    of the same elements, for throughput)."""
    m = cheb2d_mesh()
    return Workload(name="cheb2d_replicated", E=m.E * copies, nodes=np.tile(m.nodes, (copies, 1, 1)),
                    mat=np.tile(m.mat, (copies, 1)))
