"""FP64 reference of the tail statistic of the learned quadrature order.

TEST INFRASTRUCTURE ONLY (the test-suite compares the library's tail
records and decisions with it).  Shares no code with the product library.

With Q Gauss points along an axis the discrete Legendre coefficient of
degree d of a line of values y_a is
    c_d = (2d+1)/2 * sum_a w_a L_d(x_a) y_a,
which equals the exact Legendre coefficient when the line is a polynomial of
degree <= Q-1 (Gauss exactness, degree 2d <= 2Q-2).  The moment integrals of
eq. (4) of degree k < K_m = 2N-1 along an axis are exact unless the sampled
function has Legendre content of degree >= 2Q-k along it.

Per field, the record holds for each axis the envelope (largest magnitude
over lines) of c_{Q-1}, ..., c_{Q-4} and the largest magnitude of the tensor
whose lines were taken:
    axis u: lines of the samples alpha[.][b][c];
    axis v: lines of the u-moments P1[k][.][c] = sum_a W_u[k][a] alpha[a][b][c];
    axis w: lines of the (u,v)-moments P2[k][l][.] = sum_b W_v[l][b] P1[k][b][c];
with W[k][a] = w_a L_k(x_a), k, l < K_m.  An axis sampled with the full
rule (Q >= qfull) records zeros.  The element's tail value combines, over
the fields, the envelopes A_j and scale S of each reduced axis as
    r2 = min(1, max(A_1/A_3, A_2/A_4)),
    est = max(A_1, A_2) * r2 ** max(0, (Q - K_m + 2)/2),
    tau = max over reduced axes of est / S,
i.e. the top resolvable content extrapolated at its own two-degree decay to
the first degree the moments can alias.
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


def records(alpha, Qu, Qv, Qw, N, qfull=24):
    """Tail records [F][16] of one element from its coupling samples
    alpha [F][Qu*Qv*Qw] (index (a*Qv + b)*Qw + c)."""
    Km = 2 * N - 1
    F = alpha.shape[0]
    A = alpha.reshape(F, Qu, Qv, Qw)
    out = np.zeros((F, REC))
    xu, wu = _rule(Qu)
    xv, wv = _rule(Qv)
    Wu = _legendre_rows(xu, Km) * wu
    Wv = _legendre_rows(xv, Km) * wv
    for f in range(F):
        a = A[f]
        P1 = np.einsum("ka,abc->kbc", Wu, a)      # [Km][Qv][Qw]
        P2 = np.einsum("lb,kbc->klc", Wv, P1)     # [Km][Km][Qw]
        if Qu < qfull:
            c = np.einsum("ja,abc->jbc", _tail_rows(Qu), a)
            out[f, 0:4] = np.abs(c).reshape(4, -1).max(1)
            out[f, 12] = np.abs(a).max()
        if Qv < qfull:
            c = np.einsum("jb,kbc->jkc", _tail_rows(Qv), P1)
            out[f, 4:8] = np.abs(c).reshape(4, -1).max(1)
            out[f, 13] = np.abs(P1).max()
        if Qw < qfull:
            c = np.einsum("jc,klc->jkl", _tail_rows(Qw), P2)
            out[f, 8:12] = np.abs(c).reshape(4, -1).max(1)
            out[f, 14] = np.abs(P2).max()
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
