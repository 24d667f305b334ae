"""FP64 CPU oracle of the paper's 2-D example: curl-curl + mass element
matrices of a curved quadrilateral with the Chebyshev vector basis.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it; it shares no code with the product
library.

What it computes (Section III of the paper, eqs. (5)-(15)).  The field of
an element is expanded in the basis of eq. (6) on the reference square
[-1,1]^2:
    u-functions  E_u = U_m(u) T_n(v),  m = 0..M-1, n = 0..N,
    v-functions  E_v = T_m(u) U_n(v),  m = 0..M,   n = 0..N-1,
taken as covariant components (E = J^-T E_hat).  The element matrix is
    s_K * S + s_M * M,
with S and M the stiffness and mass integrals of eq. (7) written on the
reference square as in eqs. (8)-(15):
    S_tb = int curl_hat(E_t) curl_hat(E_b) / (mu_r J) du dv,
           curl_hat(E_u-function) = -n U_m(u) U_{n-1}(v),
           curl_hat(E_v-function) =  m U_{m-1}(u) U_n(v);
    M_tb = int eps_r E_hat_t^T G E_hat_b du dv,  G = [[x_v^2 + y_v^2, -(x_u x_v + y_u y_v)],
                                                     [-(x_u x_v + y_u y_v), x_u^2 + y_u^2]] / J,
where J = x_u y_v - x_v y_u.  Every integral is taken by direct tensor
Gauss-Legendre quadrature with Q points per axis (the "direct numerical
integration" the paper compares against); the product-to-sum method of eqs.
(16)-(19) reaches the same discrete sums.

Geometry: a fourth-order (25-node) Lagrange quadrilateral, node (i, j) at
index i + 5 j (i along u) at the reference point (-1 + i/2, -1 + j/2).
Material: eps_r = p0 exp(p1 x + p2 y + p3) (the paper's 2 exp(x + y + 2) is
p = (2, 1, 1, 2)); mu_r = 1.

Degrees of freedom: the M (N+1) u-functions, index m (N+1) + n, then the
(M+1) N v-functions, index M (N+1) + m N + n.  This oracle takes M = N.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

NODES1D = np.array([-1.0, -0.5, 0.0, 0.5, 1.0])


def cheb_t(nmax, x):
    """T_0..T_nmax at points x: [nmax+1][len(x)] (three-term recurrence)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((nmax + 1, x.size))
    out[0] = 1.0
    if nmax >= 1:
        out[1] = x
    for n in range(1, nmax):
        out[n + 1] = 2.0 * x * out[n] - out[n - 1]
    return out


def cheb_u(nmax, x):
    """U_0..U_nmax at points x: [nmax+1][len(x)] (three-term recurrence)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((nmax + 1, x.size))
    out[0] = 1.0
    if nmax >= 1:
        out[1] = 2.0 * x
    for n in range(1, nmax):
        out[n + 1] = 2.0 * x * out[n] - out[n - 1]
    return out


def lagrange4(t):
    """Values and derivatives of the five quartic Lagrange polynomials on
    NODES1D at points t: ([5][len(t)], [5][len(t)])."""
    t = np.asarray(t, dtype=np.float64)
    val = np.ones((5, t.size))
    der = np.zeros((5, t.size))
    for i in range(5):
        others = [j for j in range(5) if j != i]
        den = np.prod([NODES1D[i] - NODES1D[j] for j in others])
        for j in others:
            val[i] *= (t - NODES1D[j])
        val[i] /= den
        for k in others:
            term = np.ones_like(t)
            for j in others:
                if j != k:
                    term = term * (t - NODES1D[j])
            der[i] += term
        der[i] /= den
    return val, der


def num_dofs(M: int) -> int:
    return 2 * M * (M + 1)


def geometry(nodes, u, v):
    """x, y, x_u, x_v, y_u, y_v at the points (u[a], v[b]) of a tensor
    grid: each [len(u)][len(v)]."""
    X = np.asarray(nodes, dtype=np.float64).reshape(5, 5, 2)  # [j][i][r]: node i + 5 j
    lu, du = lagrange4(u)
    lv, dv = lagrange4(v)
    out = []
    for r in range(2):
        C = X[:, :, r]  # C[j][i]
        val = lu.T @ C.T @ lv          # [a][b] = sum_ij lu_i(a) C[j][i] lv_j(b)
        d_u = du.T @ C.T @ lv
        d_v = lu.T @ C.T @ dv
        out.append((val, d_u, d_v))
    (x, xu, xv), (y, yu, yv) = out
    return x, y, xu, xv, yu, yv


def element_matrix(nodes, mat, M, Q, s_K=1.0, s_M=1.0):
    """Dense element matrix [ndof][ndof] and the status bit (1 if J <= 0 at
    some Gauss point) of one element of order M = N with Q x Q points."""
    N = M
    t, w = npleg.leggauss(Q)
    x, y, xu, xv, yu, yv = geometry(nodes, t, t)
    J = xu * yv - xv * yu
    bad = bool((J <= 0).any())
    eps = mat[0] * np.exp(mat[1] * x + mat[2] * y + mat[3])
    W = np.outer(w, w)
    gS = W / J                                     # 1/(mu_r J), mu_r = 1
    g_uu = W * eps * (xv * xv + yv * yv) / J
    g_uv = -W * eps * (xu * xv + yu * yv) / J
    g_vv = W * eps * (xu * xu + yu * yu) / J
    Tt, Ut = cheb_t(M + 1, t), cheb_u(M + 1, t)
    P = Q * Q
    # reference components and curls of every basis function at every point
    nd = num_dofs(M)
    Eu = np.zeros((nd, P))   # u component
    Ev = np.zeros((nd, P))   # v component
    C = np.zeros((nd, P))    # curl_hat
    i = 0
    for m in range(M):
        for n in range(N + 1):
            Eu[i] = np.outer(Ut[m], Tt[n]).reshape(-1)
            if n >= 1:
                C[i] = -n * np.outer(Ut[m], Ut[n - 1]).reshape(-1)
            i += 1
    for m in range(M + 1):
        for n in range(N):
            Ev[i] = np.outer(Tt[m], Ut[n]).reshape(-1)
            if m >= 1:
                C[i] = m * np.outer(Ut[m - 1], Ut[n]).reshape(-1)
            i += 1
    gS, g_uu, g_uv, g_vv = (g.reshape(-1) for g in (gS, g_uu, g_uv, g_vv))
    S = (C * gS) @ C.T
    Mm = (Eu * g_uu) @ Eu.T + (Eu * g_uv) @ Ev.T + (Ev * g_uv) @ Eu.T + (Ev * g_vv) @ Ev.T
    return s_K * S + s_M * Mm, bad


def fill(nodes, mat, M, Q, s_K=1.0, s_M=1.0):
    """Element matrices of E elements: (out [E][ndof*ndof], status [E])."""
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 25, 2)
    mat = np.asarray(mat, dtype=np.float64).reshape(-1, 4)
    E = nodes.shape[0]
    nd = num_dofs(M)
    out = np.zeros((E, nd * nd))
    st = np.zeros(E, dtype=np.uint32)
    for e in range(E):
        A, bad = element_matrix(nodes[e], mat[e], M, Q, s_K, s_M)
        out[e] = A.reshape(-1)
        st[e] = 1 if bad else 0
    return out, st
