"""Pins of the 2-D Chebyshev oracle (oracle/cheb2d.py) and of the product
identities of eqs. (16)-(17), against facts fixed by the mathematics: numpy's
Chebyshev series, exact series integrals on affine elements, the exact
sequence (curl of a gradient), adaptive quadrature on a curved element,
symmetry and scaling."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import cheb2d


def t_series(n):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return c


def u_series(n):
    """U_n as a Chebyshev-T series: U_n = T'_{n+1} / (n+1)."""
    return C.chebder(t_series(n + 1)) / (n + 1)


def tns_def(n, x):
    """Eq. (17): the nonsingular Chebyshev polynomial by its definition."""
    T = C.chebval(x, t_series(n))
    return (T - 1.0) / (2 * (1 - x * x)) if n % 2 == 0 else (T - x) / (2 * (1 - x * x))


def test_recurrences_match_numpy_chebyshev():
    x = np.linspace(-1, 1, 37)
    T = cheb2d.cheb_t(20, x)
    U = cheb2d.cheb_u(20, x)
    for n in range(21):
        assert np.abs(T[n] - C.chebval(x, t_series(n))).max() < 1e-13
        assert np.abs(U[n] - C.chebval(x, u_series(n))).max() < 1e-12 * max(1, n * n)


def test_product_to_sum_identities_eq16():
    """Eq. (16) with the 1/2 factors of the T.T and U.T products, U_{-1} = 0
    and U_{-k} = -U_{k-2}; T^ns by its definition, eq. (17)."""
    rng = np.random.default_rng(0)
    x = rng.uniform(-0.95, 0.95, 64)
    T = cheb2d.cheb_t(40, x)
    U = cheb2d.cheb_u(40, x)

    def Us(k):
        return U[k] if k >= 0 else (0.0 if k == -1 else -U[-k - 2])
    for a in range(12):
        for b in range(12):
            lhs = U[a] * U[b]
            assert np.abs(lhs - (tns_def(abs(a - b), x) - tns_def(a + b + 2, x))).max() < 1e-9 * (1 + np.abs(lhs).max())
            assert np.abs(T[a] * T[b] - 0.5 * (T[abs(a - b)] + T[a + b])).max() < 1e-12
            assert np.abs(U[a] * T[b] - 0.5 * (Us(a + b) + Us(a - b))).max() < 1e-11 * (1 + a + b)


def test_nonsingular_chebyshev_recurrence_and_limits():
    """T^ns_0 = T^ns_1 = 0 and T^ns_{n+2} = T^ns_n - U_n (eq. (16) with one
    factor U_0 = 1) reproduce eq. (17) inside (-1, 1) and its limits at
    +-1: -n^2/4 (n even), -(n^2-1)/4 (n odd) at u = 1."""
    x = np.concatenate([np.linspace(-0.99, 0.99, 41), [1.0, -1.0]])
    U = cheb2d.cheb_u(40, x)
    tns = np.zeros((41, x.size))
    for n in range(2, 41):
        tns[n] = tns[n - 2] - U[n - 2]
    inner = np.abs(x) < 1
    for n in range(41):
        assert np.abs(tns[n][inner] - tns_def(n, x[inner])).max() < 1e-8 * (1 + n * n)
        lim = -(n * n) / 4 if n % 2 == 0 else -(n * n - 1) / 4
        assert abs(tns[n][-2] - lim) < 1e-9 * (1 + n * n)
        assert abs(tns[n][-1] - lim * (1 if n % 2 == 0 else -1)) < 1e-9 * (1 + n * n)


def square_nodes(A=np.eye(2), b=np.zeros(2)):
    n = np.zeros((25, 2))
    for j in range(5):
        for i in range(5):
            n[i + 5 * j] = A @ np.array([cheb2d.NODES1D[i], cheb2d.NODES1D[j]]) + b
    return n


def curved_nodes(seed, amp=0.02):
    rng = np.random.default_rng(seed)
    return square_nodes(np.diag([0.5, 0.4])) + rng.uniform(-amp, amp, (25, 2))


def exact1d(s1, s2):
    p = C.chebint(C.chebmul(s1, s2))
    return C.chebval(1.0, p) - C.chebval(-1.0, p)


@pytest.mark.parametrize("M", [2, 3, 5])
def test_affine_element_matches_exact_series_integrals(M):
    """Parallelogram, constant eps: J and the mass metric are constants, so
    every entry is a product of two exact 1-D Chebyshev-series integrals."""
    A = np.array([[0.7, 0.2], [-0.1, 0.5]])
    nodes = square_nodes(A, np.array([0.3, -0.2]))
    eps = 2.0 * math.exp(0.5)
    mat = np.array([2.0, 0.0, 0.0, 0.5])
    xu, xv, yu, yv = A[0, 0], A[0, 1], A[1, 0], A[1, 1]
    J = xu * yv - xv * yu
    Guu, Guv, Gvv = (xv * xv + yv * yv) / J, -(xu * xv + yu * yv) / J, (xu * xu + yu * yu) / J
    N = M
    T, U = t_series, u_series
    ui = [(m, n) for m in range(M) for n in range(N + 1)]
    vi = [(m, n) for m in range(M + 1) for n in range(N)]
    nd = len(ui) + len(vi)
    S = np.zeros((nd, nd))
    Mm = np.zeros((nd, nd))
    for a, (m1, n1) in enumerate(ui):
        for b, (m2, n2) in enumerate(ui):
            if n1 and n2:
                S[a, b] = n1 * n2 * exact1d(U(m1), U(m2)) * exact1d(U(n1 - 1), U(n2 - 1)) / J
            Mm[a, b] = eps * Guu * exact1d(U(m1), U(m2)) * exact1d(T(n1), T(n2))
        for b, (m2, n2) in enumerate(vi):
            bb = len(ui) + b
            if n1 and m2:
                S[a, bb] = -n1 * m2 * exact1d(U(m1), U(m2 - 1)) * exact1d(U(n1 - 1), U(n2)) / J
            Mm[a, bb] = eps * Guv * exact1d(U(m1), T(m2)) * exact1d(T(n1), U(n2))
            S[bb, a], Mm[bb, a] = S[a, bb], Mm[a, bb]
    for a, (m1, n1) in enumerate(vi):
        for b, (m2, n2) in enumerate(vi):
            aa, bb = len(ui) + a, len(ui) + b
            if m1 and m2:
                S[aa, bb] = m1 * m2 * exact1d(U(m1 - 1), U(m2 - 1)) * exact1d(U(n1), U(n2)) / J
            Mm[aa, bb] = eps * Gvv * exact1d(T(m1), T(m2)) * exact1d(U(n1), U(n2))
    got, bad = cheb2d.element_matrix(nodes, mat, M, M + 2, 1.0, 0.0)
    assert not bad
    assert np.abs(got - S).max() < 1e-12 * np.abs(S).max()
    got, _ = cheb2d.element_matrix(nodes, mat, M, M + 2, 0.0, 1.0)
    assert np.abs(got - Mm).max() < 1e-12 * np.abs(Mm).max()


@pytest.mark.parametrize("M", [2, 4])
def test_exact_sequence_on_a_curved_element(M):
    """The curl of the gradient of T_a(u) T_b(v) is zero: its coefficients
    (a on u-function (a-1, b), b on v-function (a, b-1)) span the null space
    of the stiffness matrix on any geometry and material."""
    N = M
    nodes = curved_nodes(3)
    S, _ = cheb2d.element_matrix(nodes, [2.0, 1.0, 1.0, 2.0], M, 9, 1.0, 0.0)
    nd = cheb2d.num_dofs(M)
    cols = []
    for a in range(M + 1):
        for b in range(N + 1):
            g = np.zeros(nd)
            if a >= 1:
                g[(a - 1) * (N + 1) + b] = a
            if b >= 1:
                g[M * (N + 1) + a * N + (b - 1)] = b
            if a or b:
                cols.append(g)
    G = np.array(cols).T
    assert np.abs(S @ G).max() < 1e-12 * np.abs(S).max() * np.abs(G).max()
    ev = np.linalg.eigvalsh(S)
    assert (np.abs(ev) < 1e-10 * ev.max()).sum() == (M + 1) * (N + 1) - 1


def test_symmetry_scaling_rotation():
    nodes = curved_nodes(4)
    mat0 = [1.5, 0.0, 0.0, 0.0]
    A, _ = cheb2d.element_matrix(nodes, [2.0, 1.0, 1.0, 2.0], 3, 8)
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    S, _ = cheb2d.element_matrix(nodes, mat0, 3, 8, 1.0, 0.0)
    Mm, _ = cheb2d.element_matrix(nodes, mat0, 3, 8, 0.0, 1.0)
    h = 2.5
    S2, _ = cheb2d.element_matrix(h * nodes, mat0, 3, 8, 1.0, 0.0)
    M2, _ = cheb2d.element_matrix(h * nodes, mat0, 3, 8, 0.0, 1.0)
    assert np.abs(S2 - S / h ** 2).max() < 1e-13 * np.abs(S).max()
    assert np.abs(M2 - Mm).max() < 1e-13 * np.abs(Mm).max()
    c, s = math.cos(0.7), math.sin(0.7)
    R = np.array([[c, -s], [s, c]])
    S3, _ = cheb2d.element_matrix(nodes @ R.T, mat0, 3, 8, 1.0, 0.0)
    M3, _ = cheb2d.element_matrix(nodes @ R.T, mat0, 3, 8, 0.0, 1.0)
    assert np.abs(S3 - S).max() < 1e-13 * np.abs(S).max()
    assert np.abs(M3 - Mm).max() < 1e-13 * np.abs(Mm).max()


def test_curved_element_against_adaptive_quadrature():
    """M = 1 on a curved element with the paper's material: a few entries by
    adaptive integration (scipy) of the reference-square integrands, the
    map built from scipy's Lagrange polynomials; the oracle at 40 points
    converges to them."""
    from scipy import integrate
    from scipy.interpolate import lagrange
    nodes = curved_nodes(5, 0.02)
    mat = [2.0, 1.0, 1.0, 2.0]
    ref, _ = cheb2d.element_matrix(nodes, mat, 1, 40)
    basis = [lagrange(cheb2d.NODES1D, np.eye(5)[i]) for i in range(5)]
    dbasis = [np.polyder(p) for p in basis]
    X = nodes.reshape(5, 5, 2)  # [j][i]

    def geo(u, v):
        lu = np.array([p(u) for p in basis]); du = np.array([p(u) for p in dbasis])
        lv = np.array([p(v) for p in basis]); dv = np.array([p(v) for p in dbasis])
        x, y = (lv @ X[:, :, r] @ lu for r in range(2))
        xu, yu = (lv @ X[:, :, r] @ du for r in range(2))
        xv, yv = (dv @ X[:, :, r] @ lu for r in range(2))
        return x, y, xu, xv, yu, yv

    # dofs at M = N = 1: u-functions (0,0), (0,1) = U0 T0, U0 T1; v-functions (0,0), (1,0) = T0 U0, T1 U0
    Eu = [lambda u, v: 1.0, lambda u, v: v, lambda u, v: 0.0, lambda u, v: 0.0]
    Ev = [lambda u, v: 0.0, lambda u, v: 0.0, lambda u, v: 1.0, lambda u, v: u]
    curl = [lambda u, v: 0.0, lambda u, v: -1.0, lambda u, v: 0.0, lambda u, v: 1.0]

    def integrand(v, u, i, j):
        x, y, xu, xv, yu, yv = geo(u, v)
        J = xu * yv - xv * yu
        eps = mat[0] * math.exp(mat[1] * x + mat[2] * y + mat[3])
        s = curl[i](u, v) * curl[j](u, v) / J
        m = eps * (Eu[i](u, v) * Eu[j](u, v) * (xv * xv + yv * yv) - (Eu[i](u, v) * Ev[j](u, v)
                   + Ev[i](u, v) * Eu[j](u, v)) * (xu * xv + yu * yv) + Ev[i](u, v) * Ev[j](u, v)
                   * (xu * xu + yu * yu)) / J
        return s + m
    for i, j in [(0, 0), (1, 1), (1, 3), (0, 2), (2, 3), (3, 3)]:
        val, err = integrate.dblquad(integrand, -1, 1, -1, 1, args=(i, j), epsabs=1e-13, epsrel=1e-13)
        assert abs(ref[i, j] - val) < 1e-11 * max(1.0, abs(val)), (i, j, ref[i, j], val)
