"""The allocation-free entry point p2s_fill_uniform_noalloc against the
one-shot p2s_fill_element_matrices on the same inputs, through the C ABI:
two calls in a row, the second with a smaller batch (the scratch keeps the
first call's contents), bit-identical blocks and status.  The first
workload spans several scratch chunks; the second fits in one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1703_09619_amd as p2s
    from paper_1703_09619_amd import workloads as W
    return dict(torch=torch, p2s=p2s, W=W, ctx=p2s.Context(0))


def _compare(env, w):
    torch, ctx = env["torch"], env["ctx"]
    print("case", w.name, "E", w.E, "N", int(w.orders[0]), "Q", w.quad[0].tolist(), flush=True)
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    ref, rst = ctx.fill_element_matrices(w.problem, w.material, nodes, mat, w.orders, w.quad)
    out = torch.full_like(ref, float("nan"))
    st = torch.full_like(rst, -1)
    ctx.fill_uniform_noalloc(w.problem, w.material, nodes, mat, w.E, int(w.orders[0]), w.quad[0], out, st)
    torch.cuda.synchronize()
    assert torch.equal(st, rst)
    assert torch.equal(out, ref)


def test_noalloc_matches_one_shot_two_calls(env):
    W = env["W"]
    # 300 vector N=6 elements at 12^3 points: 294 KB of scratch each, so the
    # 64 MiB scratch takes them in two chunks
    _compare(env, W.subset(W.make("vector_n6", E=300), np.arange(300)))
    # then a smaller scalar batch on the same scratch
    _compare(env, W.subset(W.make("scalar_n4"), np.arange(17)))


def test_noalloc_rejects_bad_arguments(env):
    torch, p2s, ctx = env["torch"], env["p2s"], env["ctx"]
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(p2s.P2SError, match="order"):
        ctx.fill_uniform_noalloc(0, 0, x, x, 1, 9, (4, 4, 4), x, s)
    with pytest.raises(p2s.P2SError, match="Gauss"):
        ctx.fill_uniform_noalloc(0, 0, x, x, 1, 4, (33, 4, 4), x, s)
    with pytest.raises(p2s.P2SError, match="moment stage"):
        ctx.fill_uniform_noalloc(0, 0, x, x, 1, 8, (32, 32, 32), x, s)
