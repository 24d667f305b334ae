"""FP64 reference of the tail statistic of the learned quadrature order.

TEST INFRASTRUCTURE ONLY (the test-suite compares the library's tail
records and decisions with it).  Shares no code with the product library.

What the statistic measures.  The moments of eq. (4) are taken with Q Gauss
points per axis; along an axis, the moment of degree k is exact unless the
coupling factor, seen through the moment degrees of the other two axes, has
Legendre content along that axis at degrees >= 2Q - k.  The content a
Q-point rule can still resolve is the discrete Legendre coefficient
    c_d = (2d+1)/2 * sum_a w_a L_d(x_a) y_a      (d <= Q-1),
exact for polynomial lines of degree <= Q-1.  For each axis x sampled below
the full rule, each field s and the four highest resolvable degrees
d = Q_x-1-j (j = 0..3), the statistic takes
    T_x[j] = the degree-d coefficient along x of alpha_s, projected on the
             other two axes onto the Legendre moments of degree < K_m = 2N-1,
e.g. T_u[j][l][q] = sum_{a,b,c} t_j(a) W_v[l][b] W_w[q][c] alpha_s(a,b,c)
with t_j(a) = (2d+1)/2 w_a L_d(x_a) and W[l][b] = w_b L_l(x_b).  It is the
same for every axis (no axis order is involved).  The record of a field
holds the envelopes A_x[j] = max |T_x[j][.][.]| and, for every reduced
axis, the scale S = max |I_s| of the field's moment tensor.  The element's
tail value combines them over the fields as
    r2 = min(1, max(A_0/A_2, A_1/A_3)),
    est = max(A_0, A_1) * r2 ** max(0, (Q - K_m + 2)/2),
    tau = max over reduced axes of est / S,
i.e. the top resolvable content extrapolated at its own two-degree decay to
the first degree the moments can alias.  Axes sampled with the full rule
(Q >= qfull) take no statistic: a refill could not change them.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

REC = 16


def _rule(Q):
    return npleg.leggauss(Q)


def _legendre_rows(x, kmax):
    """L_k(x_a) for k < kmax: [kmax][len(x)]."""
    out = np.zeros((kmax, len(x)))
    for k in range(kmax):
        c = np.zeros(k + 1)
        c[k] = 1.0
        out[k] = npleg.legval(x, c)
    return out


def _tail_rows(Q):
    """(2d+1)/2 w_a L_d(x_a) for d = Q-1 .. Q-4 (zero rows for d < 0)."""
    x, w = _rule(Q)
    L = _legendre_rows(x, Q)
    rows = np.zeros((4, Q))
    for j in range(4):
        d = Q - 1 - j
        if d >= 0:
            rows[j] = 0.5 * (2 * d + 1) * w * L[d]
    return rows


def _moment_rows(Q, Km):
    """w_a L_k(x_a) for k < Km: [Km][Q]."""
    x, w = _rule(Q)
    return _legendre_rows(x, Km) * w


def records(alpha, Qu, Qv, Qw, N, qfull=24):
    """Tail records [F][16] of one element from its coupling samples
    alpha [F][Qu*Qv*Qw] (index (a*Qv + b)*Qw + c): env[axis][j] at axis*4+j,
    the scale at 12+axis (zeros for axes at the full rule), 15 unused."""
    Km = 2 * N - 1
    F = alpha.shape[0]
    A = alpha.reshape(F, Qu, Qv, Qw)
    Wu, Wv, Ww = _moment_rows(Qu, Km), _moment_rows(Qv, Km), _moment_rows(Qw, Km)
    Tu, Tv, Tw = _tail_rows(Qu), _tail_rows(Qv), _tail_rows(Qw)
    out = np.zeros((F, REC))
    for f in range(F):
        a = A[f]
        S = np.abs(np.einsum("ka,lb,qc,abc->klq", Wu, Wv, Ww, a, optimize=True)).max()
        if Qu < qfull:
            T = np.einsum("ja,lb,qc,abc->jlq", Tu, Wv, Ww, a, optimize=True)
            out[f, 0:4] = np.abs(T).reshape(4, -1).max(1)
            out[f, 12] = S
        if Qv < qfull:
            T = np.einsum("ka,jb,qc,abc->jkq", Wu, Tv, Ww, a, optimize=True)
            out[f, 4:8] = np.abs(T).reshape(4, -1).max(1)
            out[f, 13] = S
        if Qw < qfull:
            T = np.einsum("ka,lb,jc,abc->jkl", Wu, Wv, Tw, a, optimize=True)
            out[f, 8:12] = np.abs(T).reshape(4, -1).max(1)
            out[f, 14] = S
    return out


def tail_value(rec, Q, N, qfull=24):
    """Element tail value from its records [F][16] and rule Q = (Qu,Qv,Qw)."""
    Km = 2 * N - 1
    tau = 0.0
    for ax in range(3):
        if Q[ax] >= qfull:
            continue
        A = rec[:, ax * 4:ax * 4 + 4].max(0)
        S = rec[:, 12 + ax].max()
        r2 = max(A[0] / A[2] if A[2] > 0 else 1.0, A[1] / A[3] if A[3] > 0 else 1.0)
        r2 = min(r2, 1.0)
        est = max(A[0], A[1]) * r2 ** max(0.0, 0.5 * (Q[ax] - Km + 2))
        tau = max(tau, est / max(S, 1e-300))
    return tau
