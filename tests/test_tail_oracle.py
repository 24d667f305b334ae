"""Pins of the FP64 tail-statistic reference (oracle/tail.py): closed forms
of the discrete Legendre transform on products of Legendre polynomials
(exact by Gauss exactness and orthogonality, int L_d^2 = 2/(2d+1)), and
properties of the element tail value."""
import numpy as np
from numpy.polynomial import legendre as npleg

from oracle import tail


def legendre_product_field(Qu, Qv, Qw, i, j, d):
    def L(k, x):
        c = np.zeros(k + 1)
        c[k] = 1.0
        return npleg.legval(x, c)
    xu, _ = npleg.leggauss(Qu)
    xv, _ = npleg.leggauss(Qv)
    xw, _ = npleg.leggauss(Qw)
    f = L(i, xu)[:, None, None] * L(j, xv)[None, :, None] * L(d, xw)[None, None, :]
    return f.reshape(1, -1), L(i, xu), L(j, xv)


def test_records_of_a_legendre_product():
    Qu, Qv, Qw, N = 12, 10, 14, 8           # K_m = 15 covers every degree used
    i, j, d = Qu - 2, Qv - 1, Qw - 3
    alpha, _, Lj = legendre_product_field(Qu, Qv, Qw, i, j, d)
    r = tail.records(alpha, Qu, Qv, Qw, N)[0]
    xw, _ = npleg.leggauss(Qw)
    c = np.zeros(d + 1)
    c[d] = 1.0
    Ld = np.abs(npleg.legval(xw, c)).max()
    m_jd = np.abs(Lj).max() * Ld
    cu, cv = 2.0 / (2 * i + 1), 2.0 / (2 * j + 1)
    tol = 1e-13
    # u: only degree Qu-2 is present, coefficient L_j L_d on every line
    assert np.allclose(r[0:4], [0, m_jd, 0, 0], atol=tol, rtol=1e-12)
    assert abs(r[12] - np.abs(alpha).max()) <= tol
    # v: the u-moments are cu * L_j L_d at k = i only; degree Qv-1 on b
    assert np.allclose(r[4:8], [cu * Ld, 0, 0, 0], atol=tol, rtol=1e-12)
    assert abs(r[13] - cu * m_jd) <= tol
    # w: the (u,v)-moments are cu*cv*L_d at (k,l) = (i,j) only; degree Qw-3
    assert np.allclose(r[8:12], [0, 0, cu * cv, 0], atol=tol, rtol=1e-12)
    assert abs(r[14] - cu * cv * Ld) <= tol
    assert r[15] == 0.0


def test_full_axes_record_nothing():
    alpha, _, _ = legendre_product_field(24, 9, 24, 3, 8, 5)
    r = tail.records(alpha, 24, 9, 24, 6)[0]
    assert (r[0:4] == 0).all() and (r[8:12] == 0).all() and r[12] == 0 and r[14] == 0
    assert r[4] > 0 and r[13] > 0


def test_tail_value_properties():
    rng = np.random.default_rng(3)
    Q, N = (14, 9, 24), 6
    # low-degree polynomial along the reduced axes: no content at the top degrees
    alpha, _, _ = legendre_product_field(*Q, Q[0] - 5, Q[1] - 5, 7)
    rec = tail.records(alpha + 2.0, *Q, N)
    assert tail.tail_value(rec, Q, N) <= 1e-14
    # scale invariance, and a larger top coefficient raises the value
    base = rng.standard_normal((2, Q[0] * Q[1] * Q[2]))
    t1 = tail.tail_value(tail.records(base, *Q, N), Q, N)
    t2 = tail.tail_value(tail.records(3.7 * base, *Q, N), Q, N)
    assert abs(t1 - t2) <= 1e-12 * t1
    spike, _, _ = legendre_product_field(*Q, Q[0] - 1, 0, 0)
    t3 = tail.tail_value(tail.records(base + 50.0 * spike, *Q, N), Q, N)
    assert t3 > t1
    # nothing reduced -> zero
    full = (24, 24, 24)
    assert tail.tail_value(tail.records(base[:, :1].repeat(24 ** 3, 1), *full, N), full, N) == 0.0
