"""GPU parity of the paper's 2-D Chebyshev example (p2s_cheb2d_*) against
the oracle's direct quadrature (oracle/cheb2d.py) on the stand-in mesh of
the paper's Fig. 2, through the C ABI: the product-to-sum form (eqs.
(16)-(19)) and the direct form, orders 1..18.  Bar: relative Frobenius error
<= 1e-10 per element (eq. (16) is an exact identity, so both forms reach
the oracle's discrete sums up to rounding)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1703_09619_amd as p2s
    from oracle import cheb2d
    from paper_1703_09619_amd import workloads as W
    return dict(torch=torch, p2s=p2s, cheb2d=cheb2d, W=W, ctx=p2s.Context(0))


def run(env, w, M, Q, method, sK=1.0, sM=1.0):
    torch = env["torch"]
    print("case E", w.E, "M", M, "Q", Q, "method", method, flush=True)
    c = env["ctx"].cheb2d(w.E, M, Q)
    out, st = c.execute(torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda(), method, sK, sM)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(w.E, -1), st.cpu().numpy()


def check(env, w, M, Q, method, sK=1.0, sM=1.0):
    got, st = run(env, w, M, Q, method, sK, sM)
    ref, rst = env["cheb2d"].fill(w.nodes, w.mat, M, Q, sK, sM)
    assert (st == rst.astype(st.dtype)).all()
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print("max rel err %.3e" % err.max(), flush=True)
    assert err.max() <= TOL
    return got


@pytest.mark.parametrize("M,Q", [(1, 3), (2, 5), (3, 7), (4, 8), (6, 10), (8, 14), (12, 18), (18, 24), (18, 32)])
def test_product_to_sum_and_direct_against_oracle(env, M, Q):
    w = env["W"].cheb2d_mesh()
    if M >= 12:
        w = env["W"].subset(w, np.array([0, 5, 10, 15]))
    a = check(env, w, M, Q, env["p2s"].METHOD_P2S)
    b = check(env, w, M, Q, env["p2s"].METHOD_DIRECT)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


def test_scales_and_symmetry(env):
    w = env["W"].cheb2d_mesh()
    p2s = env["p2s"]
    check(env, w, 5, 9, p2s.METHOD_P2S, 1.0, 0.0)
    check(env, w, 5, 9, p2s.METHOD_P2S, 0.0, 1.0)
    got = check(env, w, 5, 9, p2s.METHOD_P2S, 1.0, -3.0)
    nd = 2 * 5 * 6
    A = got.reshape(w.E, nd, nd)
    assert np.abs(A - A.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(A).max()


def test_inverted_element_and_arguments(env):
    W, p2s, torch = env["W"], env["p2s"], env["torch"]
    w = W.subset(W.cheb2d_mesh(), np.arange(3))
    w["nodes"] = w.nodes.copy()
    w["nodes"][1, 12] = (5.0, 5.0)  # centre node far outside: tangled map
    _, st = run(env, w, 3, 6, p2s.METHOD_P2S)
    assert st[1] & p2s.STATUS_DETJ and st[0] == 0 and st[2] == 0
    with pytest.raises(p2s.P2SError):
        env["ctx"].cheb2d(4, 19, 8)
    with pytest.raises(p2s.P2SError):
        env["ctx"].cheb2d(4, 3, 33)
