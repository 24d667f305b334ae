"""CPU-side tests of the product library: the C ABI loads and exports every
declared symbol, and its host tables (Gauss rules, linearization of eq. (3))
are right.  No kernel runs here."""
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def p2s():
    import paper_1703_09619_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1703_09619_amd import build
        build.build()
    m.load()
    return m


def header_functions():
    src = open(os.path.join(ROOT, "include", "p2s.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(p2s_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(p2s):
    lib = p2s.load()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(p2s.EXPORTS) == names


def test_num_dofs_and_layout(p2s):
    assert p2s.num_dofs(p2s.SCALAR, 4) == 64
    assert p2s.num_dofs(p2s.VECTOR, 6) == 540
    assert p2s.num_dofs(p2s.VECTOR, 8) == 1344
    assert p2s.num_dofs(p2s.SCALAR, 1) == -1
    assert p2s.num_dofs(p2s.SCALAR, 9) == -1
    off = p2s.layout(p2s.SCALAR, [2, 4, 3])
    assert off.tolist() == [0, 64, 64 + 4096, 64 + 4096 + 729]
    with pytest.raises(p2s.P2SError):
        p2s.layout(p2s.VECTOR, [6, 11])


def test_packed_layout(p2s):
    off = p2s.layout(p2s.VECTOR, [6, 2, 3], p2s.OUTPUT_PACKED_UPPER)
    sizes = [540 * 541 // 2, 12 * 13 // 2, 54 * 55 // 2]
    assert off.tolist() == [0, sizes[0], sizes[0] + sizes[1], sum(sizes)]
    with pytest.raises(p2s.P2SError):
        p2s.layout(p2s.SCALAR, [3], 7)


def test_create_without_device_fails_cleanly(p2s):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(p2s.P2SError, match="no HIP device"):
        p2s.Context(0)


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 7, 12, 16, 24, 32])
def test_gauss_rule(p2s, Q):
    x, w = p2s.gauss_rule(Q)
    xr, wr = npleg.leggauss(Q)
    assert np.abs(x - xr).max() < 4e-15 and np.abs(w - wr).max() < 4e-15
    with pytest.raises(p2s.P2SError):
        p2s.gauss_rule(33)


def test_linearization_matches_golden_rationals(p2s):
    """Legendre products (psi_m = sqrt((2m+1)/2) L_m) against exact rational
    expansions from tests/golden/legendre_products.txt."""
    path = os.path.join(ROOT, "tests", "golden", "legendre_products.txt")
    for line in open(path):
        if line.startswith("#"):
            continue
        a, b, k, n, d = map(int, line.split())
        c = p2s.linearization(p2s.FAM_PSI, a, p2s.FAM_PSI, b)
        scale = math.sqrt((2 * a + 1) / 2) * math.sqrt((2 * b + 1) / 2)
        assert abs(c[k] / scale - n / d) < 1e-15


def _series(kind, m):
    if kind == 0:  # phi
        if m == 0:
            return np.array([0.5, -0.5])
        if m == 1:
            return np.array([0.5, 0.5])
        c = np.zeros(m + 1)
        c[m], c[m - 2] = 1.0, -1.0
        return c / math.sqrt(2 * (2 * m - 1))
    if kind == 1:  # phi'
        return npleg.legder(_series(0, m)) if m >= 1 else np.array([-0.5])
    c = np.zeros(m + 1)
    c[m] = math.sqrt((2 * m + 1) / 2)
    return c


@pytest.mark.parametrize("xf", [0, 1, 2])
@pytest.mark.parametrize("yf", [0, 1, 2])
def test_linearization_is_exact_product(p2s, xf, yf):
    """sum_k C[k] L_k(t) == X_m1(t) Y_m2(t) (numpy Legendre series), and the
    expansion agrees with the Gauss projection (2k+1)/2 int X Y L_k."""
    rng = np.random.default_rng(0)
    t = rng.uniform(-1, 1, 50)
    xg, wg = npleg.leggauss(20)
    for m1 in range(8):
        for m2 in range(8):
            if (xf == 2 and m1 == 7) or (yf == 2 and m2 == 7):
                continue
            c = p2s.linearization(xf, m1, yf, m2)
            sx, sy = _series(xf, m1), _series(yf, m2)
            lhs = npleg.legval(t, c)
            rhs = npleg.legval(t, sx) * npleg.legval(t, sy)
            assert np.abs(lhs - rhs).max() < 2e-14
            prod = npleg.legval(xg, sx) * npleg.legval(xg, sy)
            for k in range(16):
                proj = (2 * k + 1) / 2 * np.sum(wg * prod * npleg.legval(xg, np.eye(k + 1)[k]))
                assert abs(proj - c[k]) < 2e-14 * (2 * k + 1) * max(1.0, np.abs(prod).max())
            # degree rule of eq. (3): the highest degree is m1+m2 minus one
            # per derivative factor
            deg = (m1 if xf == 0 else m1 - 1 if xf == 1 else m1) + (m2 if yf == 0 else m2 - 1 if yf == 1 else m2)
            if xf == 0 and m1 < 2:
                deg = deg - m1 + 1
            if yf == 0 and m2 < 2:
                deg = deg - m2 + 1
            if xf == 1 and m1 < 2:
                deg = deg - (m1 - 1)
            if yf == 1 and m2 < 2:
                deg = deg - (m2 - 1)
            assert np.all(c[deg + 1:] == 0.0)


def test_linearization_sparsity(p2s):
    """The tables are sparse (the paper ties efficiency to this, Section II):
    a same-family Legendre product has at most min(m1,m2)+1 terms of one
    parity."""
    for m1 in range(7):
        for m2 in range(7):
            c = p2s.linearization(2, m1, 2, m2)
            nz = np.nonzero(c)[0]
            assert len(nz) == min(m1, m2) + 1
            assert np.all((nz - (m1 + m2)) % 2 == 0)
