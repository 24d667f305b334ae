"""GPU tests of the split forms (moment and contraction products on the
FP32 matrix cores on exact 10-bit operand slices, or on the INT8 matrix
cores on exact 7-bit slices; FP64 coupling, tables, intermediates and
sums) against the CPU oracle and the FP64 GPU path.

Bar: relative Frobenius error <= 1e-8 per element, the precision target of
the split form.  Every FP32 matrix-core sum is exact (integer slice
products below 2^20, at most 16 per sum); what is left is the dropped
slice products of order >= 4 and the last slice's rounding, about 2^-40
relative per product, so observed errors sit near 1e-11."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BOUND = 1e-8


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1703_09619_amd as p2s
    from paper_1703_09619_amd import workloads as W
    oracle.build(force=False)
    return dict(torch=torch, oracle=oracle, p2s=p2s, W=W, ctx=p2s.Context(0))


def small(W, problem, N, E, Q, seed):
    rng = np.random.default_rng(seed)
    nodes, _, _ = W.perturbed_nodes(rng, E, 0.12)
    if problem == W.SCALAR:
        material, mat = W.MAT_SINCOSEXP, rng.uniform(math.pi, 4 * math.pi, size=(E, 1))
    else:
        material = W.MAT_ROTDIAG
        mat = np.zeros((E, 12))
        for e in range(E):
            mat[e, :9] = W.haar_rotation(rng).reshape(-1)
        mat[:, 9:] = W.unit_vectors(rng, E) * rng.uniform(0, 4 * math.pi, (E, 1))
    return W.Workload(name="small", problem=problem, material=material, E=E, nodes=nodes, mat=mat,
                      orders=np.full(E, N, np.int32), quad=np.tile(np.array(Q, np.int32), (E, 1)))


def fill(env, w, precision):
    torch = env["torch"]
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad, precision=precision)
    out, st = plan.execute(torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan.offsets, st.cpu().numpy()


def rel(a, b, off):
    return np.array([np.linalg.norm(a[off[e]:off[e + 1]] - b[off[e]:off[e + 1]]) /
                     np.linalg.norm(b[off[e]:off[e + 1]]) for e in range(len(off) - 1)])


PRECISIONS = ("SPLIT_FP32", "SPLIT_INT8")


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("problem,N,Q", [(0, 4, (8, 8, 8)), (0, 6, (12, 10, 9)), (1, 3, (6, 6, 6)),
                                         (1, 5, (10, 9, 11)), (0, 8, (16, 16, 16)), (0, 2, (3, 4, 5))])
def test_split_against_oracle(env, problem, N, Q, prec):
    W, oracle, p2s = env["W"], env["oracle"], env["p2s"]
    w = small(W, problem, N, 3, Q, seed=100 + 10 * N + problem)
    print("case problem %d N %d Q %s %s" % (problem, N, Q, prec), flush=True)
    out, off, st = fill(env, w, getattr(p2s, prec))
    ref, roff, rst = oracle.fill(w.problem, w.material, w.nodes, w.mat, w.orders, w.quad)
    assert np.array_equal(off, roff) and (st == 0).all()
    err = rel(out, ref, off)
    print("split-FP32 vs oracle: max rel Frobenius %.3e" % err.max(), flush=True)
    assert err.max() <= BOUND
    # symmetric: mirrored blocks are copies; the diagonal slabs (m1 = m2) are
    # computed whole, so their two triangles differ by the slice error only
    for e in range(w.E):
        n = int(round(math.sqrt(off[e + 1] - off[e])))
        M = out[off[e]:off[e + 1]].reshape(n, n)
        assert np.linalg.norm(M - M.T) <= BOUND * np.linalg.norm(M)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_split_vector_n8_against_oracle(env, prec):
    """The precision configuration: vector curl-curl + mass at N = 8 with
    16^3 points (1344 dofs), eight elements of the 8192-element workload
    (first, last and six between) against the oracle, and the same elements
    through the FP64 GPU path."""
    W, oracle, p2s = env["W"], env["oracle"], env["p2s"]
    full = W.make("vector_n8")
    idx = np.array([0, 1, 1000, 2500, 4096, 6000, 8000, 8191])
    w = W.subset(full, idx)
    out, off, st = fill(env, w, getattr(p2s, prec))
    out64, _, _ = fill(env, w, p2s.FP64)
    ref, roff, _ = oracle.fill(w.problem, w.material, w.nodes, w.mat, w.orders, w.quad)
    e_split, e_64 = rel(out, ref, off), rel(out64, ref, off)
    print("vector N=8: %s max %.3e, FP64 max %.3e" % (prec, e_split.max(), e_64.max()), flush=True)
    assert (st == 0).all()
    assert e_64.max() <= 1e-10
    assert e_split.max() <= BOUND


@pytest.mark.parametrize("prec", PRECISIONS)
def test_split_moments_against_fp64(env, prec):
    W, p2s, torch = env["W"], env["p2s"], env["torch"]
    w = small(W, 1, 6, 4, (12, 12, 12), seed=7)
    nodes, mat = torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda()
    m32 = env["ctx"].plan(w.problem, w.material, w.orders, w.quad,
                          precision=getattr(p2s, prec)).moments(nodes, mat)
    m64 = env["ctx"].plan(w.problem, w.material, w.orders, w.quad).moments(nodes, mat)
    a, b = m32.cpu().numpy(), m64.cpu().numpy()
    err = np.linalg.norm((a - b).reshape(w.E, -1), axis=1) / np.linalg.norm(b.reshape(w.E, -1), axis=1)
    print("moments split vs FP64: %.3e" % err.max(), flush=True)
    assert err.max() <= BOUND / 2


def test_split_argument_errors(env):
    p2s = env["p2s"]
    ctx = env["ctx"]
    with pytest.raises(p2s.P2SError, match="split-FP32"):
        ctx.plan(0, 0, [4, 4], [[8, 8, 8], [8, 8, 9]], precision=p2s.SPLIT_FP32)
    with pytest.raises(p2s.P2SError, match="split-FP32"):
        ctx.plan(0, 0, [4], [[17, 8, 8]], precision=p2s.SPLIT_FP32)
    with pytest.raises(p2s.P2SError, match="split-FP32"):
        ctx.plan(0, 0, [4], [[8, 8, 8]], precision=p2s.SPLIT_FP32, method=p2s.METHOD_DIRECT)
    with pytest.raises(p2s.P2SError, match="split-INT8"):
        ctx.plan(0, 0, [4], [[17, 8, 8]], precision=p2s.SPLIT_INT8)
