"""Pins of the FP64 tail-statistic reference (oracle/tail.py): closed forms
of the projected discrete Legendre coefficients on products of Legendre
polynomials (exact by Gauss exactness and orthogonality, int L_d^2 =
2/(2d+1)), the axis symmetry of the definition, and properties of the
element tail value."""
import numpy as np
from numpy.polynomial import legendre as npleg

from oracle import tail


def L(k, x):
    c = np.zeros(k + 1)
    c[k] = 1.0
    return npleg.legval(x, c)


def product_field(Q, fu, fv, fw):
    """alpha = fu(u) fv(v) fw(w) at the tensor Gauss points, [1][P]."""
    xs = [npleg.leggauss(q)[0] for q in Q]
    f = fu(xs[0])[:, None, None] * fv(xs[1])[None, :, None] * fw(xs[2])[None, None, :]
    return f.reshape(1, -1)


def test_records_of_a_legendre_product():
    """alpha = (1 + L_i(u)) (1 + L_j(v)) (1 + L_d(w)) with the top-degree
    terms at i = Qu-2, j = Qv-1, d = Qw-3 and N = 4 (moment degrees < 7):
    every discrete product used is Gauss-exact, so the moments are 8 at
    (0,0,0) and 0 elsewhere, and along each axis only the coefficient of its
    own top-degree term survives, projected onto the constant moment 2 of
    each other axis: envelope 4 at position Q-1-deg."""
    Qu, Qv, Qw, N = 12, 10, 14, 4
    i, j, d = Qu - 2, Qv - 1, Qw - 3
    alpha = product_field((Qu, Qv, Qw), lambda x: 1 + L(i, x), lambda x: 1 + L(j, x), lambda x: 1 + L(d, x))
    r = tail.records(alpha, Qu, Qv, Qw, N)[0]
    tol = 1e-12
    assert np.allclose(r[0:4], [0, 4, 0, 0], atol=tol)    # u: degree Qu-2 -> j = 1
    assert np.allclose(r[4:8], [4, 0, 0, 0], atol=tol)    # v: degree Qv-1 -> j = 0
    assert np.allclose(r[8:12], [0, 0, 4, 0], atol=tol)   # w: degree Qw-3 -> j = 2
    assert np.allclose(r[12:15], [8, 8, 8], atol=tol)
    assert r[15] == 0.0


def test_projection_uses_the_other_axes_moments():
    """alpha = L_i(u) L_1(v): the u-tail is the coefficient 1 times the
    v-moment of L_1 (2/3 at degree 1) times the w-moment of 1 (2); a v
    factor of degree >= K_m (not a moment degree) projects to zero."""
    Q, N = (9, 8, 7), 3                   # K_m = 5
    a1 = product_field(Q, lambda x: L(Q[0] - 1, x), lambda x: L(1, x), lambda x: np.ones_like(x))
    r = tail.records(a1, *Q, N)[0]
    assert np.allclose(r[0:4], [2.0 / 3.0 * 2.0, 0, 0, 0], atol=1e-13)
    a2 = product_field(Q, lambda x: L(Q[0] - 1, x), lambda x: L(5, x), lambda x: np.ones_like(x))
    r2 = tail.records(a2, *Q, N)[0]
    assert np.abs(r2[0:4]).max() <= 1e-13


def test_definition_is_symmetric_in_the_axes():
    """Permuting the axes of the field and the rule permutes the records:
    no axis order enters the definition."""
    rng = np.random.default_rng(4)
    Q, N = (9, 11, 7), 4
    a = rng.standard_normal(Q)
    r = tail.records(a.reshape(1, -1), *Q, N)[0]
    perm = (2, 0, 1)                       # new axis k is old axis perm[k]
    ap = np.transpose(a, perm)
    Qp = tuple(Q[p] for p in perm)
    rp = tail.records(ap.reshape(1, -1), *Qp, N)[0]
    for k in range(3):
        assert np.allclose(rp[4 * k:4 * k + 4], r[4 * perm[k]:4 * perm[k] + 4], rtol=1e-12, atol=1e-14)
    assert np.allclose(rp[12:15], r[12:15], rtol=1e-13)


def test_full_axes_record_nothing():
    alpha = product_field((24, 9, 24), lambda x: 1 + L(3, x), lambda x: 1 + L(8, x), lambda x: 1 + L(5, x))
    r = tail.records(alpha, 24, 9, 24, 6)[0]
    assert (r[0:4] == 0).all() and (r[8:12] == 0).all() and r[12] == 0 and r[14] == 0
    assert r[4] > 0 and r[13] > 0


def test_tail_value_properties():
    rng = np.random.default_rng(3)
    Q, N = (14, 9, 24), 6
    # low-degree polynomial along the reduced axes: no content at the top degrees
    alpha = product_field(Q, lambda x: 2 + L(Q[0] - 5, x), lambda x: 1 + L(Q[1] - 5, x), lambda x: L(7, x))
    rec = tail.records(alpha, *Q, N)
    assert tail.tail_value(rec, Q, N) <= 1e-14
    # scale invariance, and a larger top coefficient raises the value
    base = rng.standard_normal((2, Q[0] * Q[1] * Q[2]))
    t1 = tail.tail_value(tail.records(base, *Q, N), Q, N)
    t2 = tail.tail_value(tail.records(3.7 * base, *Q, N), Q, N)
    assert abs(t1 - t2) <= 1e-12 * t1
    spike = product_field(Q, lambda x: L(Q[0] - 1, x), lambda x: np.ones_like(x), lambda x: np.ones_like(x))
    t3 = tail.tail_value(tail.records(base + 50.0 * spike, *Q, N), Q, N)
    assert t3 > t1
    # nothing reduced -> zero
    full = (24, 24, 24)
    assert tail.tail_value(tail.records(base[:, :1].repeat(24 ** 3, 1), *full, N), full, N) == 0.0
